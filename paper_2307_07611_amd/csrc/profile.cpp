// Launch profiling (measurement helper): when enabled, every profiled launch
// scope of the library gets a pair of HIP events carried by its kernel
// dispatches, together with its algorithmic flops and bytes. The pairs are
// resolved (and the GPU waited for) only when the profile is read.
#include "profile.h"

#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace trinv {

namespace {
struct Rec {
  std::string cls;
  double flops, bytes;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::set<std::string> g_select;  // empty: every class
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local ProfLaunch* tl_scope = nullptr;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool profiling_on() { return g_on; }

ProfLaunch::ProfLaunch(const char* cls, double flops, double bytes, hipStream_t s) : s_(s) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_select.empty() && !g_select.count(cls)) return;
  Rec r;
  r.cls = cls;
  r.flops = flops;
  r.bytes = bytes;
  r.a = get_event();
  r.b = get_event();
  if (!r.a || !r.b) return;
  g_recs.push_back(r);
  a_ = r.a;
  b_ = r.b;
  outer_ = tl_scope;
  tl_scope = this;
}

ProfLaunch::~ProfLaunch() {
  if (!a_) return;
  tl_scope = outer_;
  if (launched_ == 0) {  // nothing launched: an empty interval
    (void)hipEventRecord(a_, s_);
    (void)hipEventRecord(b_, s_);
  }
}

LaunchEvents next_launch_events() {
  ProfLaunch* p = tl_scope;
  if (!p) return LaunchEvents{nullptr, nullptr};
  LaunchEvents e{p->launched_ == 0 ? p->a_ : nullptr, p->b_};
  ++p->launched_;
  return e;
}

}  // namespace trinv

using namespace trinv;

extern "C" int trinv_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return TRINV_OK;
}

extern "C" int trinv_profile_select(const char* classes) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_select.clear();
  if (!classes) return TRINV_OK;
  std::string cur;
  for (const char* p = classes;; ++p) {
    if (*p == ',' || *p == '\0') {
      if (!cur.empty()) g_select.insert(cur);
      cur.clear();
      if (*p == '\0') break;
    } else {
      cur.push_back(*p);
    }
  }
  return TRINV_OK;
}

extern "C" int trinv_profile_read(trinv_profile_entry* out, int max_entries) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, trinv_profile_entry> agg;
  std::vector<std::string> order;
  for (Rec& r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -TRINV_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -TRINV_ERR_HIP;
    auto it = agg.find(r.cls);
    if (it == agg.end()) {
      trinv_profile_entry e;
      std::memset(&e, 0, sizeof(e));
      std::strncpy(e.name, r.cls.c_str(), sizeof(e.name) - 1);
      it = agg.emplace(r.cls, e).first;
      order.push_back(r.cls);
    }
    it->second.launches += 1;
    it->second.total_ms += ms;
    it->second.flops += r.flops;
    it->second.bytes += r.bytes;
  }
  int n = 0;
  for (const std::string& k : order) {
    if (n < max_entries && out) out[n] = agg[k];
    ++n;
  }
  return n;
}
