// Low-precision MFMA tile products (BF16 or FP16 inputs, FP32 accumulation)
// for the mixed-precision path: the off-diagonal products of the recursion
// (Section 4.1, algorithm COMBRIT with beta = 2) and the products of the
// Newton-Schulz refinement (not in the paper).
//
// Tiling for gfx950: a 256-thread workgroup computes a 256 x 256 tile with
// v_mfma_f32_32x32x16_{bf16,f16}; each wave owns a 128 x 128 sub-tile
// (4 x 4 blocks of 32 x 32, 256 FP32 accumulators per lane). Both operands
// are k-contiguous in memory (B is stored transposed), so a K step is staged
// by direct global -> LDS 16-byte loads into a ring of LDS stages (at most
// 160 KB: five of K = 32 for the single products, five or six of K = 16 for
// the 2- and 3-product residuals), issued one stage short of the ring ahead, and
// every MFMA operand is one 16-byte LDS read. Lane
// layouts (measured on gfx950): lane l supplies A(l%32, 8(l/32)+e) and
// B(8(l/32)+e, l%32), e = 0..7, and receives D(8(r/4) + 4(l/32) + r%4, l%32)
// in register r.
//
// The optional 3-product split forms A_hi B_hi + A_hi B_lo + A_lo B_hi in the
// same accumulator (an operand v is carried as hi = round(v) plus
// lo = round(v - hi), which multiplies the precision by the slice width); the
// 2-product form A_hi B_hi + A_lo B_hi serves a B that its hi slice holds
// exactly.
// Rows beyond M (columns beyond N) are clamped to the last valid one: they
// only feed outputs that are not stored. Zero fill beyond K and the element
// masks of triangular operands are applied only in K steps that reach the K
// edge or a masked diagonal.
#include <type_traits>

#include "common.h"
#include "lowp.h"

namespace trinv {

namespace {
constexpr int LT = 256;  // workgroup tile (rows and columns)
constexpr int kTrLd = LT + 8;  // row length of a transposed tile staged in LDS (16-byte rows, fewer bank conflicts)
// Residual epilogue staging in LDS (after the main loop): diagonals of L and
// X at kEpDiagOff (4 KB), per-wave X / L blocks at kEpStageOff (128 KB); the
// first bytes hold the final reduction.
constexpr int kEpDiagOff = 1024, kEpStageOff = 8192, kEpLdsBytes = kEpStageOff + 4 * 4 * 8192;

// K per LDS stage: 16 (one MFMA k step) for the 2- and 3-product residuals
// on panel-blocked planes, whose loads are spread over the MFMAs of the
// stage before and run four or five stages ahead; 32 for the other products.
constexpr int lp_kt(int nsplit, int klo) { return (klo == kLoN0Pb && nsplit >= 2) ? 16 : 32; }

template <int NSPLIT, int KT_>
struct LpShape {
  static constexpr int KT = KT_;
  static constexpr int NT = NSPLIT == 1 ? 2 : (NSPLIT == 2 ? 3 : 4);  // staged tiles per stage
  static constexpr int CPR = KT / 8;                // 16-byte chunks per tile row
  static constexpr int TILE = LT * KT;              // elements of one staged tile (no padding)
  static constexpr int RPI = 512 / KT;              // tile rows per 1 KB direct-load instruction
  static constexpr int IPW = KT / 8;                // direct-load instructions per wave per tile
  static constexpr int LPS = NT * IPW;              // direct loads per thread and stage
  static constexpr int RSW = 128 / KT;              // rows per swizzle step
  // LDS stages (at most 160 KB, at most 5 of K = 32 or 8 of K = 16, and at
  // most 63 loads of newer stages outstanding per thread): loads run
  // NBUF - 1 stages ahead
  static constexpr int NB_LDS = 163840 / (NT * LT * KT * 2);
  static constexpr int NB_VM = 1 + 63 / LPS;
  static constexpr int NB_MAX = KT == 16 ? 8 : 5;
  static constexpr int NBUF = NB_LDS < NB_VM ? (NB_LDS < NB_MAX ? NB_LDS : NB_MAX) : (NB_VM < NB_MAX ? NB_VM : NB_MAX);
  static_assert(NBUF >= 2, "two stages at least");
  static_assert(KT == 16 || KT == 32, "one or two MFMA k steps per stage");
  // Chunk position p of row r holds the row's k-chunk p ^ swz(r): 16
  // consecutive rows read at one logical chunk hit 16 distinct bank groups.
  static __device__ __forceinline__ int swz(int r) { return (r / RSW) % CPR; }
  static_assert(32 % (RSW * CPR) == 0, "swizzle period must divide the 32-row fragment block");
};

typedef unsigned short u16;
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int F16>
__device__ __forceinline__ f32x16 mma(u32x4 a, u32x4 b, f32x16 c) {
  if (F16) return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Waits (gfx9 s_waitcnt encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8) followed by a workgroup barrier, with no memory fence: the
// direct global -> LDS loads of newer stages stay in flight across it. VM is
// the number of this wave's direct loads allowed to remain outstanding; all
// its LDS reads are complete, so buffers read before the barrier may be
// refilled after it.
template <int VM>
__device__ __forceinline__ void wait_barrier() {
  static_assert(VM >= 0 && VM < 64, "vmcnt range");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4));  // lgkmcnt(0), vmcnt(VM)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int F16>
__device__ __forceinline__ u16 to_lp(float v) {
  if (F16) return __builtin_bit_cast(u16, (_Float16)v);
  return __builtin_bit_cast(u16, (__bf16)v);
}

template <int F16>
__device__ __forceinline__ float lp_to_f32(u16 v) {
  if (F16) return (float)__builtin_bit_cast(_Float16, v);
  return (float)__builtin_bit_cast(__bf16, v);
}

__device__ __forceinline__ int64_t tri_root_lp(int64_t q) {
  int64_t u = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (u * (u + 1) / 2 > q) --u;
  while ((u + 1) * (u + 2) / 2 <= q) ++u;
  return u;
}

template <int TILES, int ORDER>
__device__ __forceinline__ void decode_lp(int64_t t, int64_t nz, int64_t tm, int64_t tn, int64_t& z, int64_t& it,
                                          int64_t& jt) {
  if (TILES == kAllTiles) {
    if (ORDER == kRowDesc) {
      const int64_t g = t / (nz * tn), r = t % (nz * tn);
      it = tm - 1 - g;
      z = r / tn;
      jt = r % tn;
    } else {
      const int64_t g = t / (nz * tm), r = t % (nz * tm);
      jt = g;
      z = r / tm;
      it = r % tm;
    }
    return;
  }
  const int64_t per = tm * (tm + 1) / 2;
  z = t / per;
  const int64_t q = t % per;
  const int64_t u = tri_root_lp(q), w = q - u * (u + 1) / 2;
  jt = w;  // kDiagDesc: offset it - jt descending
  it = w + (tm - 1 - u);
}

// Element masks (A(m,k): 1 lower k<=m, 2 strict k<m; B(k,n): 1 lower k>=n, 2 strict k>n).
template <int MASK, bool IS_A>
__device__ __forceinline__ bool lp_mask_ok(int64_t r, int64_t k) {
  if (MASK == 0) return true;
  if (IS_A) return MASK == 1 ? (k <= r) : (k < r);
  return MASK == 1 ? (k >= r) : (k > r);
}
}  // namespace

int64_t gemm_lp_tiles(const GemmBatch& bt, int tiles) {
  const int64_t tm = (bt.M + LT - 1) / LT, tn = (bt.N + LT - 1) / LT;
  if (tiles == kLowerTiles) return bt.nmerge * tm * (tm + 1) / 2;
  return bt.nmerge * tm * tn;
}

template <int F16, int NSPLIT, int AM, int BM, int TILES, int ORDER, int KLO, int KHI, int EPI>
__global__ __launch_bounds__(256) void k_gemm_lp(LpGemmArgs a) {
  typedef LpShape<NSPLIT, lp_kt(NSPLIT, KLO)> S;
  constexpr int KT = S::KT;
  // NBUF stages x NT tiles x TILE elements (all of the CU's LDS); after the
  // main loop its first bytes hold the per-wave partial sums of the residual
  extern __shared__ __attribute__((aligned(16))) u16 lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  const GemmBatch bt = a.bt;
  const int64_t tm = (bt.M + LT - 1) / LT, tn = (bt.N + LT - 1) / LT;
  const int64_t nz = bt.nmerge;
  // L2-aware schedule: tiles are grouped in GB x GB blocks run by 16
  // consecutive workgroups of one XCD (workgroups are dispatched round-robin
  // over the 8 XCDs), so a block's tiles share GB row panels and GB column
  // panels in that XCD's L2. Blocks are taken heaviest first, eight per round,
  // and the rounds alternate direction over the XCDs (round r gives block
  // 8r + x to XCD x when r is even, 8r + 7 - x when odd), so that no XCD
  // receives the heaviest block of every round.
  constexpr int GB = 4;
  const int64_t bm = (tm + GB - 1) / GB, bn = (tn + GB - 1) / GB;
  const int64_t nblk = (TILES == kLowerTiles) ? nz * bm * (bm + 1) / 2 : nz * bm * bn;
  const int64_t w = blockIdx.x, x = w % kNumXcd, q = w / kNumXcd;
  const int64_t round = q / (GB * GB);
  const int64_t B = round * kNumXcd + ((round & 1) ? kNumXcd - 1 - x : x);
  const int pos = (int)(q % (GB * GB));
  if (B >= nblk) return;
  int64_t z, bi, bj;
  decode_lp<TILES, ORDER>(B, nz, bm, bn, z, bi, bj);
  // the decode runs on vector instructions; its results are wave-uniform,
  // and scalar copies keep the tile's address and stage bookkeeping scalar
  z = __builtin_amdgcn_readfirstlane((int)z);
  bi = __builtin_amdgcn_readfirstlane((int)bi);
  bj = __builtin_amdgcn_readfirstlane((int)bj);
  const int64_t it = bi * GB + pos % GB, jt = bj * GB + pos / GB;
  // slot of this tile in the per-tile partial sums (lower tiles packed)
  const int64_t t = (TILES == kLowerTiles) ? z * tm * (tm + 1) / 2 + it * (it + 1) / 2 + jt : (z * tm + it) * tn + jt;
  if (it >= tm || jt >= tn) return;
  if (TILES == kLowerTiles && it < jt) return;
  const bool last = (z == bt.nmerge - 1);
  const int64_t M = last ? bt.M_last : bt.M, N = last ? bt.N_last : bt.N, K = last ? bt.K_last : bt.K;
  const int64_t m0 = it * LT, n0 = jt * LT;
  if (m0 >= M || n0 >= N) {
    if (EPI == kLpEpResid && tid == 0) {
      a.tile_sq[t] = 0.0;
      a.tile_sqx[t] = 0.0;
    }
    return;
  }
  int64_t klo = 0, khi = K;
  if (KLO == kLoN0) klo = n0;
  if (KLO == kLoN0Pb) klo = n0;
  if (KHI == kHiM1) khi = imin64(K, m0 + LT);
  klo = (klo / KT) * KT;

  // Staging by direct global -> LDS loads: instruction i of wave w fills
  // tile rows [q RPI, (q+1) RPI), q = w IPW + i; lane L writes 16 bytes at
  // LDS byte L*16 of that 1 KB block, i.e. row q RPI + L / CPR, chunk position
  // L % CPR, and so loads the row's k-chunk (L % CPR) ^ swz(row). Rows beyond
  // M (N) are clamped; they only feed outputs that are not stored.
  const u16* tb[4];
  tb[0] = (const u16*)a.A_hi + z * a.a_bstride;
  tb[1] = (const u16*)a.Bt_hi + z * a.b_bstride;
  tb[2] = NSPLIT >= 2 ? (const u16*)a.A_lo + z * a.a_bstride : nullptr;
  tb[3] = NSPLIT == 3 ? (const u16*)a.Bt_lo + z * a.b_bstride : nullptr;
  // Panel-blocked operands (refinement products): the stage of a tile is
  // KT / 16 consecutive 8 KB blocks of its 256-row panel, copied linearly, so
  // the LDS tile is [KT / 16][256][16] with the plane's half exchange.
  // The tile's first source element (its row or panel base at klo) goes into
  // the 64-bit base pointer; the per-lane offsets stay inside one 256-row
  // panel (below 256 ld elements), so they fit 32 bits for any order whose
  // planes the host accepts.
  constexpr bool PB = (KLO == kLoN0Pb);
  uint32_t off[S::NT][S::IPW];  // byte offsets of this lane's source chunk from tb[tt], stage 0
#pragma unroll
  for (int tt = 0; tt < S::NT; ++tt) {
    const bool isb = tt & 1;
    const int64_t ld = isb ? a.ldb : a.lda;
    const int64_t r0 = isb ? n0 : m0, rmax = (isb ? N : M) - 1;
    tb[tt] += PB ? ((r0 >> 8) * ld + (klo >> 4)) * 4096 : r0 * ld + klo;
#pragma unroll
    for (int i = 0; i < S::IPW; ++i) {
      if constexpr (PB) {
        off[tt][i] = (uint32_t)(((wave * S::IPW + i) * 512 + lane * 8) * 2);
      } else {
        const int row = (wave * S::IPW + i) * S::RPI + lane / S::CPR;
        const int chunk = (lane % S::CPR) ^ S::swz(row);
        const int64_t grow = imin64(r0 + row, rmax);
        off[tt][i] = (uint32_t)(((grow - r0) * ld + 8 * chunk) * 2);
      }
    }
  }
  // direct load i of tile tt of the stage starting at klo + kstage, into buffer buf
  auto issue_one = [&](int buf, int64_t kstage, int tt, int i) __attribute__((always_inline)) {
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* base = (lds_char*)lds + (size_t)buf * S::NT * S::TILE * 2;
    const char* src = (const char*)tb[tt] + (PB ? (kstage >> 4) * 4096 * 2 : kstage * 2);
    __builtin_amdgcn_global_load_lds((const void*)(src + off[tt][i]),
                                     (__attribute__((address_space(3))) void*)(base + tt * S::TILE * 2 +
                                                                               (wave * S::IPW + i) * 1024),
                                     16, 0, 0);
  };
  auto issue = [&](int buf, int64_t kstage) {  // loads of the stage starting at klo + kstage
#pragma unroll
    for (int tt = 0; tt < S::NT; ++tt)
#pragma unroll
      for (int i = 0; i < S::IPW; ++i) issue_one(buf, kstage, tt, i);
  };
  // Fragment of tile tt for block blk at k step ks (16 wide): 8 elements of
  // one tile row, read from its swizzled chunk position.
  // The swizzle has a period of 16 rows, which divides 32, so it depends on
  // lane & 31 only and the block offset folds into an immediate.
  const int fsw = S::swz(lane & 31);
  const int fpb = ((lane & 31) >> 3) & 1;  // blocked layout: half exchange of the row
  auto frag = [&](const u16* base, int tt, int ks, int blk) -> u32x4 {
    const int row = ((tt & 1) ? wn : wm) * 128 + blk * 32 + (lane & 31);
    if constexpr (PB)
      return *(const u32x4*)(base + tt * S::TILE + (ks >> 4) * 4096 + row * 16 + 8 * ((lane >> 5) ^ fpb));
    const int chunk = ks / 8 + (lane >> 5);
    return *(const u32x4*)(base + tt * S::TILE + row * S::KT + 8 * (chunk ^ fsw));
  };
  // Zero fill beyond K and the element masks, applied to a staged buffer in
  // LDS (only for stages that reach the K edge or a masked diagonal): thread
  // handles 16-byte chunk positions of the tiles.
  auto mask_lds = [&](int buf, int64_t k0) {
    u16* base = lds + buf * (S::NT * S::TILE);
    constexpr int CH = LT * S::CPR;  // chunk positions per tile
#pragma unroll
    for (int tt = 0; tt < S::NT; ++tt) {
      const bool isb = tt & 1;
      const int64_t r0 = isb ? n0 : m0;
      for (int c = tid; c < CH; c += 256) {
        int row, p;
        int64_t kb;
        u32x4* ptr;
        if constexpr (PB) {  // chunk c: block c / 512, row (c / 2) % 256, half c % 2
          row = (c >> 1) & 255;
          p = c & 1;
          kb = k0 + 16 * (c >> 9) + 8 * (p ^ ((row >> 3) & 1));
          ptr = (u32x4*)(base + tt * S::TILE + 8 * c);
        } else {
          row = c / S::CPR;
          p = c % S::CPR;
          kb = k0 + 8 * (p ^ S::swz(row));
          ptr = (u32x4*)(base + tt * S::TILE + row * S::KT + 8 * p);
        }
        u32x4 v = *ptr;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = kb + e;
          const bool ok =
              (k < K) && (isb ? lp_mask_ok<BM, false>(r0 + row, k) : lp_mask_ok<AM, true>(r0 + row, k));
          const unsigned sh = 16 * (e & 1);
          v[e >> 1] &= (ok ? 0xffffffffu : ~(0xffffu << sh));
        }
        *ptr = v;
      }
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // Fragments: fr[KS slot + ks][tile][block], two slots (stage parity) of KS
  // k steps each. Products of a k step (A tile x B tile): A_hi B_hi (1);
  // A_lo B_hi, A_hi B_hi (2); A_hi B_lo, A_lo B_hi, A_hi B_hi (3).
  constexpr int KS = S::KT / 16, NT = S::NT, MF = 16 * NSPLIT, RD = 4 * NT;
  static_assert(KS * NT <= 4, "two slots of fragments fit in 128 registers");
  u32x4 fr[2 * KS][NT][4];
  auto prod_a = [](int p) constexpr { return NSPLIT == 1 ? 0 : (NSPLIT == 2 ? (p == 0 ? 2 : 0) : (p == 1 ? 2 : 0)); };
  auto prod_b = [](int p) constexpr { return NSPLIT == 3 ? (p == 0 ? 3 : 1) : 1; };
  // fragment reads [LO, HI) of a stage's KS RD (k step, then tile, block) into slot f
  auto freads = [&](const u16* base, auto FI, auto LOI, auto HII) __attribute__((always_inline)) {
    constexpr int f = decltype(FI)::value;
    static_for<decltype(LOI)::value, decltype(HII)::value>([&](auto RI) {
      constexpr int r = decltype(RI)::value, ks = r / RD, rr = r % RD;
      fr[f * KS + ks][rr / 4][rr % 4] = frag(base, rr / 4, 16 * ks, rr % 4);
    });
  };
  // MFMAs [LO, HI) of a stage's KS MF (k step, then product, i, j) from slot f
  auto mmas = [&](auto FI, auto LOI, auto HII) __attribute__((always_inline)) {
    constexpr int f = decltype(FI)::value;
    static_for<decltype(LOI)::value, decltype(HII)::value>([&](auto MI) {
      constexpr int m = decltype(MI)::value, ks = m / MF, mm = m % MF, p = mm / 16, i = (mm / 4) % 4, j = mm % 4;
      acc[i][j] = mma<F16>(fr[f * KS + ks][prod_a(p)][i], fr[f * KS + ks][prod_b(p)][j], acc[i][j]);
    });
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;

  // NBUF-stage pipeline: stage st lives in buffer st % NBUF; the loads of
  // stage st + NBUF go into the buffer stage st leaves free.
  constexpr int NBUF = S::NBUF;
  constexpr int LPS = S::LPS;
  if (klo < khi) {
    const int nst = __builtin_amdgcn_readfirstlane((int)((khi - klo + S::KT - 1) / S::KT));
    // Stage order. The tiles of a block (panel-blocked products) share row
    // and column panels but start K at their own diagonal offsets; so that
    // the tiles sharing a panel read the same k at the same time (and the
    // panel is fetched once into the XCD's L2), each tile first runs
    // ascending from the block's common start s (n0 of its last tile
    // column) to its own end, then descending from s to its own start:
    // stage st covers K from klo + kpos(st).
    int a_s = 0;
    if constexpr (PB) {
      const int64_t s0 = imin64(bj * GB + GB - 1, tn - 1) * LT;
      a_s = s0 <= klo ? 0 : (int)imin64((s0 - klo) / S::KT, nst);
    }
    auto kpos = [&](int st) -> int64_t {
      return (int64_t)S::KT * (st < nst - a_s ? a_s + st : nst - 1 - st);
    };
    auto guard_mask = [&](int st) __attribute__((always_inline)) {
      const int64_t k0 = klo + kpos(st);
      bool guard = (k0 + S::KT > K);
      if (AM != 0 && k0 + S::KT > m0 && k0 < m0 + LT) guard = true;
      if (BM != 0 && k0 + S::KT > n0 && k0 < n0 + LT) guard = true;
      if (guard) {
        mask_lds(st % NBUF, k0);
        wait_barrier<LPS * (NBUF - 1)>();  // LDS writes of the mask visible (loads stay in flight)
      }
    };
    auto stage_base = [&](int st) { return lds + (st % NBUF) * (NT * S::TILE); };
    // Step st opens with the barrier after which stage st + 1 is readable and
    // every wave has read stage st; then the KS MF MFMAs of stage st run
    // interleaved with the fragment reads of stage st + 1 and the direct
    // loads of stage st + NBUF into the buffer stage st leaves free (issued in
    // one burst, those loads would hold up the MFMAs queued behind them).
    // Every step issues its loads (beyond the last stage they repeat it, into
    // a buffer no stage reads), so exactly NBUF - 2 newer stages are
    // outstanding at each barrier. Steps go in pairs, one fragment slot each;
    // an odd count starts with a step on zero fragments (its products add
    // exact zeros), so that no MFMA sits in a branch.
    auto load_stage = [&](int q) __attribute__((always_inline)) {
      issue(q % NBUF, kpos(q < nst ? q : nst - 1));
    };
    auto open_step = [&](int st) __attribute__((always_inline)) {
      wait_barrier<(NBUF - 2) * LPS>();
      if (st + 1 < nst) guard_mask(st + 1);
    };
    auto step = [&](int st, auto FI) __attribute__((always_inline)) {
      using FN = std::integral_constant<int, 1 - decltype(FI)::value>;
      open_step(st);
      const u16* nb = stage_base(st + 1);
      const int q = st + NBUF;
      const int64_t kq = kpos(q < nst ? q : nst - 1);
      // chunk g: direct load g, its share of the fragment reads and of the
      // MFMAs, fenced so that the loads stay spread over the MFMAs
      static_for<0, LPS>([&](auto G) {
        constexpr int g = decltype(G)::value;
        issue_one(q % NBUF, kq, g / S::IPW, g % S::IPW);
        freads(nb, FN{}, std::integral_constant<int, KS * RD * g / LPS>{},
               std::integral_constant<int, KS * RD * (g + 1) / LPS>{});
        mmas(FI, std::integral_constant<int, KS * MF * g / LPS>{}, std::integral_constant<int, KS * MF * (g + 1) / LPS>{});
        __builtin_amdgcn_sched_barrier(0);
      });
    };
#pragma unroll
    for (int p = 0; p < NBUF - 1; ++p) load_stage(p);
    if (nst & 1) {
#pragma unroll
      for (int f = 0; f < KS; ++f)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
          for (int b = 0; b < 4; ++b) fr[f][tt][b] = u32x4{0u, 0u, 0u, 0u};
    } else {
      open_step(-1);
      freads(stage_base(0), I0{}, I0{}, std::integral_constant<int, KS * RD>{});
      load_stage(NBUF - 1);
    }
    for (int st = -(nst & 1); st < nst; st += 2) {
      step(st, I0{});
      step(st + 1, I1{});
    }
    wait_barrier<0>();
  }

  // ---------------------------------------------------------------- epilogues
  const bool full = (m0 + LT <= M) && (n0 + LT <= N);
  const double alpha = a.alpha;
  double sq = 0.0, sqx = 0.0;
  // arrays only read by the residual (X, L, diagonals) or by the correction
  // (R32, diagonal of X): no store of the kernel aliases them
  const double* __restrict__ Xr = a.X;
  const double* __restrict__ Lr = a.L;
  const double* __restrict__ dLr = a.dL;
  const double* __restrict__ dXr = a.dX;
  const float* __restrict__ R32r = a.R32;
  // Interior residual tile with 16-byte aligned X and L: each wave stages
  // the FP64 X and L elements of its 32 x 32 blocks in LDS by direct loads,
  // one block ahead (two slots per wave, free after the main loop), so that
  // a block's loads are in flight while the previous block is computed and
  // stored; the diagonals of L (tile rows) and X (tile columns) are staged
  // once. Same arithmetic and order as the block-by-block form below.
  const bool staged = EPI == kLpEpResid && full &&
                      ((((uintptr_t)a.X) | ((uintptr_t)a.L) | (uintptr_t)(a.ldx * 8) | (uintptr_t)(a.ldl * 8)) & 15) == 0;
  double* const dls = (double*)((char*)lds + kEpDiagOff);  // dL[m0 + r], r < 256
  double* const dxs = dls + LT;                            // dX[n0 + c], c < 256
  // T and X21: alpha and lp_scale are powers of two within the FP32 range
  // (checked at launch), so the scalings are exact and the low-precision
  // values round the FP32 accumulator times one FP32 factor (the same value
  // as rounding the FP64 product), and dividing by lp_scale is multiplying
  // by its reciprocal.
  const float alpha_f = (float)alpha, lp_f = (float)(alpha * a.lp_scale);
  const double inv_scale = 1.0 / a.lp_scale;
  // X21: the lane's first element (row m0 + wm 128 + 4 (lane / 32), column
  // n0 + wn 128 + lane % 32) in the FP64 and the low-precision copy
  double* x21x = nullptr;
  u16* x21l = nullptr;
  if constexpr (EPI == kLpEpX21) {
    const int64_t r0 = m0 + wm * 128 + 4 * (lane >> 5), c0 = n0 + wn * 128 + (lane & 31);
    x21x = a.X + z * a.x_bstride + r0 * a.ldx + c0;
    x21l = (u16*)a.Xlp + z * a.xlp_bstride + r0 * a.ldxlp + c0;
  }
  // direct loads of block b of this wave into slot b % 2: [slot][X, L][32 rows][32 doubles]
  auto fetch = [&](auto BI) __attribute__((always_inline)) {
    constexpr int b = decltype(BI)::value, i = b / 4, j = b % 4, sl = b & 1;
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* const dst = (lds_char*)lds + kEpStageOff + (wave * 4 + 2 * sl) * 8192;
    const int64_t r0b = m0 + wm * 128 + i * 32 + (lane >> 4), c0b = n0 + wn * 128 + j * 32 + (lane & 15) * 2;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      __builtin_amdgcn_global_load_lds((const void*)(Xr + (r0b + 4 * t) * a.ldx + c0b),
                                       (__attribute__((address_space(3))) void*)(dst + t * 1024), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(Lr + (r0b + 4 * t) * a.ldl + c0b),
                                       (__attribute__((address_space(3))) void*)(dst + 8192 + t * 1024), 16, 0, 0);
    }
  };
  if constexpr (EPI == kLpEpResid) {
    if (staged) {
      dls[tid] = dLr[m0 + tid];
      dxs[tid] = dXr[n0 + tid];
      __syncthreads();
      fetch(std::integral_constant<int, 0>{});
    }
  }
  // Interior correction tile: the lane's X and R elements through per-lane
  // base pointers (row m0 + wm 128 + 4 (lane / 32), column n0 + wn 128 +
  // lane % 32; uniform offsets per element), the diagonal of X for the tile's
  // rows staged in LDS once, and each block's X and R loads issued one block
  // ahead into registers (slot b % 2), so that they are in flight while the
  // previous block is computed and stored.
  double* cxw = nullptr;
  const float* crp = nullptr;
  double cx[2][16];
  float cr[2][16];
  auto cload = [&](auto BI) __attribute__((always_inline)) {
    constexpr int b = decltype(BI)::value, i = b / 4, j = b % 4, sl = b & 1;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = i * 32 + 8 * (k >> 2) + (k & 3);
      cx[sl][k] = cxw[r * a.ldx + j * 32];
      cr[sl][k] = crp[r * a.ldr + j * 32];
    }
  };
  if constexpr (EPI == kLpEpCorr) {
    if (full) {
      const int64_t r0 = m0 + wm * 128 + 4 * (lane >> 5), c0 = n0 + wn * 128 + (lane & 31);
      cxw = a.X + r0 * a.ldx + c0;
      crp = R32r + r0 * a.ldr + c0;
      dls[tid] = dXr[m0 + tid];
      __syncthreads();
      cload(std::integral_constant<int, 0>{});
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, 16>([&](auto IJ) {
        constexpr int b = decltype(IJ)::value, i = b / 4, j = b % 4, sl = b & 1;
        const f32x16 blk = acc[i][j];
        // the next block's loads stay behind this block's (vector memory
        // operations complete in order, so waiting for these does not wait
        // for those)
        if constexpr (b + 1 < 16) cload(std::integral_constant<int, b + 1>{});
        __builtin_amdgcn_sched_barrier(0);
        const int cl = wn * 128 + j * 32 + (lane & 31), rl = wm * 128 + i * 32 + 4 * (lane >> 5);
        const int64_t col = n0 + cl, rbase = m0 + rl;
        double xn[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int r = 8 * (k >> 2) + (k & 3);
          const double v = cx[sl][k] + dls[rl + r] * (double)cr[sl][k] + alpha * (double)blk[k];
          xn[k] = col <= rbase + r ? v : 0.0;
          cxw[(i * 32 + r) * a.ldx + j * 32] = xn[k];
        }
        if constexpr (!F16) {
          if (a.Xn_tb_hi) {  // uniform: the next residual's slices of the new X, from these values
            u16 hi[16], lo[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
              const double v = col < rbase + 8 * (k >> 2) + (k & 3) ? xn[k] : 0.0;  // strictly lower part
              const __bf16 h = (__bf16)v;
              const __bf16 l = (__bf16)(v - (double)(float)h);
              hi[k] = __builtin_bit_cast(u16, h);
              lo[k] = __builtin_bit_cast(u16, l);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // B role: (col, rows row0 .. row0 + 3), 8 contiguous bytes
              const int64_t e = pb_index(col, rbase + 8 * q, a.kbx);
              uint2 vh, vl;
              vh.x = (unsigned)hi[4 * q] | ((unsigned)hi[4 * q + 1] << 16);
              vh.y = (unsigned)hi[4 * q + 2] | ((unsigned)hi[4 * q + 3] << 16);
              vl.x = (unsigned)lo[4 * q] | ((unsigned)lo[4 * q + 1] << 16);
              vl.y = (unsigned)lo[4 * q + 2] | ((unsigned)lo[4 * q + 3] << 16);
              *(uint2*)((u16*)a.Xn_tb_hi + e) = vh;
              *(uint2*)((u16*)a.Xn_tb_lo + e) = vl;
            }
            if (m0 + wm * 128 + i * 32 == n0 + wn * 128 + j * 32) {  // uniform: a block on the diagonal
#pragma unroll
              for (int k = 0; k < 16; ++k)
                if (rbase + 8 * (k >> 2) + (k & 3) == col) a.dXn[col] = xn[k];
            }
          }
        }
      });
      return;
    }
  }
  static_for<0, 16>([&](auto IJ) {
      constexpr int i = decltype(IJ)::value / 4, j = decltype(IJ)::value % 4;
      const f32x16 blk = acc[i][j];
      const int64_t col = n0 + wn * 128 + j * 32 + (lane & 31);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // 4 consecutive rows per lane: r = 4q + (0..3)
        const int64_t row0 = m0 + wm * 128 + i * 32 + 8 * q + 4 * (lane >> 5);
        const bool colok = full || col < N;
        if (EPI == kLpEpT) {
          u16 o[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = to_lp<F16>(blk[4 * q + e] * alpha_f);
          uint2 v;
          v.x = (unsigned)o[0] | ((unsigned)o[1] << 16);
          v.y = (unsigned)o[2] | ((unsigned)o[3] << 16);
          *(uint2*)(lds + (col - n0) * kTrLd + (row0 - m0)) = v;  // transposed tile, stored below
        } else if (EPI == kLpEpX21) {
          u16 o[4];
          double xo[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = to_lp<F16>(blk[4 * q + e] * lp_f);
          if (a.x_round) {
#pragma unroll
            for (int e = 0; e < 4; ++e) xo[e] = (double)lp_to_f32<F16>(o[e]) * inv_scale;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) xo[e] = alpha * (double)blk[4 * q + e];
          }
          // element (i * 32 + 8 q + e, j * 32) of the lane's part: the offset is uniform
          if (full) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int64_t r = i * 32 + 8 * q + e;
              x21x[r * a.ldx + j * 32] = xo[e];
              x21l[r * a.ldxlp + j * 32] = o[e];
            }
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int64_t r = i * 32 + 8 * q + e;
              if (colok && row0 + e < M) {
                x21x[r * a.ldx + j * 32] = xo[e];
                x21l[r * a.ldxlp + j * 32] = o[e];
              }
            }
          }
          uint2 v;
          v.x = (unsigned)o[0] | ((unsigned)o[1] << 16);
          v.y = (unsigned)o[2] | ((unsigned)o[3] << 16);
          *(uint2*)(lds + (col - n0) * kTrLd + (row0 - m0)) = v;  // transposed tile, stored below
        }
      }
      if constexpr (EPI == kLpEpResid) {
        if (staged) {
          constexpr int b = decltype(IJ)::value, sl = b & 1;
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (b + 1 < 16) fetch(std::integral_constant<int, b + 1>{});
          __builtin_amdgcn_sched_barrier(0);
          // This block's 16 loads done. Vector memory operations complete in
          // issue order; issued after them: the previous block's 16 R32
          // stores (and 4 Rt stores, then waited for too) and the next
          // block's 16 loads.
          constexpr int VM = (b + 1 < 16 ? 16 : 0) + (b >= 1 ? 16 : 0);
          asm volatile("" ::: "memory");
          __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (15 << 8));
          asm volatile("" ::: "memory");
          const double* xsl = (const double*)((char*)lds + kEpStageOff + (wave * 4 + 2 * sl) * 8192);
          const double* lsl = xsl + 1024;
          const int cl = wn * 128 + j * 32 + (lane & 31), rl = wm * 128 + i * 32 + 4 * (lane >> 5);
          const int64_t col = n0 + cl, rbase = m0 + rl;
          // all LDS reads of the block first, then the arithmetic
          const double xjj = dxs[cl];
          double xv[16], ov[16], dv[16], rv[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const int lrow = 4 * (lane >> 5) + 8 * (k >> 2) + (k & 3);
            xv[k] = xsl[lrow * 32 + (lane & 31)];
            ov[k] = lsl[lrow * 32 + (lane & 31)];
            dv[k] = dls[rl + 8 * (k >> 2) + (k & 3)];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const int64_t row = rbase + 8 * (k >> 2) + (k & 3);
            const bool ok = col <= row;
            const double v =
                (row == col) ? fma(-dv[k], xv[k], 1.0) : -(alpha * (double)blk[k]) - dv[k] * xv[k] - ov[k] * xjj;
            rv[k] = ok ? v : 0.0;
            a.R32[row * a.ldr + col] = (float)rv[k];
            sq += rv[k] * rv[k];
            sqx += ok ? xv[k] * xv[k] : 0.0;
          }
          if (a.Rt) {  // uniform: the FP16 path writes R in low precision in a separate pass
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              u16 o[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) o[e] = to_lp<F16>((float)(rv[4 * q + e] * a.lp_scale));
              uint2 v;
              v.x = (unsigned)o[0] | ((unsigned)o[1] << 16);
              v.y = (unsigned)o[2] | ((unsigned)o[3] << 16);
              *(uint2*)((u16*)a.Rt + pb_index(col, rbase + 8 * q, a.ldrt)) = v;
            }
          }
          return;
        }
      }
      if constexpr (EPI == kLpEpResid || EPI == kLpEpCorr) {
        const int64_t rbase = m0 + wm * 128 + i * 32 + 4 * (lane >> 5);
        if (full) {
          // Interior tile: every (row, col) of the block lies inside the
          // matrix, so every load and store is unconditional and elements
          // above the diagonal (diagonal tiles only) are selected to zero.
          // Branches around single stores would make each store wait for
          // all earlier memory operations, earlier stores included.
          double xv[16], dv[16], ov[16];
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int k = 4 * q + e;
              const int64_t row = rbase + 8 * q + e;
              if constexpr (EPI == kLpEpResid) {
                xv[k] = Xr[row * a.ldx + col];
                ov[k] = Lr[row * a.ldl + col];
                dv[k] = dLr[row];
              } else {
                xv[k] = a.X[row * a.ldx + col];
                ov[k] = (double)R32r[row * a.ldr + col];
                dv[k] = dXr[row];
              }
            }
          if constexpr (EPI == kLpEpResid) {
            const double xjj = dXr[col];
            double rv[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
              const int64_t row = rbase + 8 * (k >> 2) + (k & 3);
              const bool ok = col <= row;
              const double v = (row == col) ? fma(-dv[k], xv[k], 1.0)
                                            : -(alpha * (double)blk[k]) - dv[k] * xv[k] - ov[k] * xjj;
              rv[k] = ok ? v : 0.0;
              a.R32[row * a.ldr + col] = (float)rv[k];
              sq += rv[k] * rv[k];
              sqx += ok ? xv[k] * xv[k] : 0.0;
            }
            if (a.Rt) {  // uniform: the FP16 path writes R in low precision in a separate pass
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                u16 o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = to_lp<F16>((float)(rv[4 * q + e] * a.lp_scale));
                uint2 v;
                v.x = (unsigned)o[0] | ((unsigned)o[1] << 16);
                v.y = (unsigned)o[2] | ((unsigned)o[3] << 16);
                *(uint2*)((u16*)a.Rt + pb_index(col, rbase + 8 * q, a.ldrt)) = v;
              }
            }
          } else {  // kLpEpCorr: X <- X + D_X R + alpha acc (exact zeros above the diagonal)
            double xn[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
              const int64_t row = rbase + 8 * (k >> 2) + (k & 3);
              const double v = xv[k] + dv[k] * ov[k] + alpha * (double)blk[k];
              xn[k] = col <= row ? v : 0.0;
              a.X[row * a.ldx + col] = xn[k];
            }
            if constexpr (!F16) {
              if (a.Xn_tb_hi) {  // uniform: the next residual's slices of the new X, from these values
                u16 hi[16], lo[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                  const int64_t row = rbase + 8 * (k >> 2) + (k & 3);
                  const double v = col < row ? xn[k] : 0.0;  // strictly lower part
                  const __bf16 h = (__bf16)v;
                  const __bf16 l = (__bf16)(v - (double)(float)h);
                  hi[k] = __builtin_bit_cast(u16, h);
                  lo[k] = __builtin_bit_cast(u16, l);
                  if (row == col) a.dXn[row] = xn[k];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {  // B role: (col, rows row0 .. row0 + 3), 8 contiguous bytes
                  const int64_t e = pb_index(col, rbase + 8 * q, a.kbx);
                  uint2 vh, vl;
                  vh.x = (unsigned)hi[4 * q] | ((unsigned)hi[4 * q + 1] << 16);
                  vh.y = (unsigned)hi[4 * q + 2] | ((unsigned)hi[4 * q + 3] << 16);
                  vl.x = (unsigned)lo[4 * q] | ((unsigned)lo[4 * q + 1] << 16);
                  vl.y = (unsigned)lo[4 * q + 2] | ((unsigned)lo[4 * q + 3] << 16);
                  *(uint2*)((u16*)a.Xn_tb_hi + e) = vh;
                  *(uint2*)((u16*)a.Xn_tb_lo + e) = vl;
                }
              }
            }
          }
          return;
        }
        // Edge tile: gather the block's FP64 / FP32 operands first, all loads
        // unconditional (out-of-triangle lanes read element 0 and discard
        // it), so that they are in flight together; then compute and store.
        const bool colok = col < N;
        double xv[16], dv[16], ov[16];
        bool okv[16];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int k = 4 * q + e;
            const int64_t row = rbase + 8 * q + e;
            okv[k] = (full || (colok && row < M)) && col <= row;
            const int64_t rr = okv[k] ? row : 0, cc = okv[k] ? col : 0;
            if constexpr (EPI == kLpEpResid) {
              xv[k] = Xr[rr * a.ldx + cc];
              ov[k] = Lr[rr * a.ldl + cc];
              dv[k] = dLr[rr];
            } else {
              xv[k] = a.X[rr * a.ldx + cc];
              ov[k] = (double)R32r[rr * a.ldr + cc];
              dv[k] = dXr[rr];
            }
          }
        if constexpr (EPI == kLpEpResid) {
          const double xjj = colok ? dXr[col] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t row0 = rbase + 8 * q;
            u16 o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int k = 4 * q + e;
              const int64_t row = row0 + e;
              double rv = 0.0;
              if (okv[k]) {
                if (row == col)
                  rv = fma(-dv[k], xv[k], 1.0);
                else
                  rv = -(alpha * (double)blk[k]) - dv[k] * xv[k] - ov[k] * xjj;
                a.R32[row * a.ldr + col] = (float)rv;
                sq += rv * rv;
                sqx += xv[k] * xv[k];
              }
              o[e] = to_lp<F16>((float)(rv * a.lp_scale));
            }
            if (a.Rt) {  // uniform: the FP16 path writes R in low precision in a separate pass
              // Rt panel-blocked (row = col, k = row0 .. row0 + 3: 8 contiguous bytes)
              u16* dst = (u16*)a.Rt + pb_index(col, row0, a.ldrt);
              if (full || (colok && row0 + 3 < M)) {
                uint2 v;
                v.x = (unsigned)o[0] | ((unsigned)o[1] << 16);
                v.y = (unsigned)o[2] | ((unsigned)o[3] << 16);
                *(uint2*)dst = v;
              } else if (colok) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  if (row0 + e < M) dst[e] = o[e];
              }
            }
          }
        } else {  // kLpEpCorr: X <- X + D_X R + alpha acc
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int k = 4 * q + e;
              const int64_t row = rbase + 8 * q + e;
              if (okv[k]) a.X[row * a.ldx + col] = xv[k] + dv[k] * ov[k] + alpha * (double)blk[k];
            }
        }
      }
    });

  if constexpr (EPI == kLpEpT || EPI == kLpEpX21) {
    // The tile's transposed low-precision output, staged in LDS (row r of it
    // is column n0 + r of the product), leaves in 16-byte pieces of its rows.
    __syncthreads();
    u16* const Tb = EPI == kLpEpT ? (u16*)a.Ot + z * a.ot_bstride : (u16*)a.Xlpt + z * a.xlpt_bstride;
    const int64_t ldt = EPI == kLpEpT ? a.ldot : a.ldxlpt;
    const bool al16 = ((((uintptr_t)Tb) | (uintptr_t)(ldt * 2)) & 15) == 0;
    for (int c = tid; c < LT * (LT / 8); c += 256) {
      const int r = c / (LT / 8), p = (c % (LT / 8)) * 8;
      if (n0 + r >= N) continue;
      u16* d = Tb + (n0 + r) * ldt + m0 + p;
      const u16* sp = lds + r * kTrLd + p;
      if (al16 && m0 + p + 8 <= M) {
        *(u32x4*)d = *(const u32x4*)sp;
      } else {
        for (int e = 0; e < 8; ++e)
          if (m0 + p + e < M) d[e] = sp[e];
      }
    }
  }
  if (EPI == kLpEpResid) {
    double(*red)[4] = (double(*)[4])lds;  // free: every wave has left the main loop (its last barrier)
    for (int m = 32; m >= 1; m >>= 1) {
      sq += __shfl_xor(sq, m, 64);
      sqx += __shfl_xor(sqx, m, 64);
    }
    if (lane == 0) {
      red[0][wave] = sq;
      red[1][wave] = sqx;
    }
    __syncthreads();
    if (tid == 0) {
      a.tile_sq[t] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      a.tile_sqx[t] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
  }
}

// Workgroups to launch: 16 per 4 x 4 tile block, blocks rounded up to a
// multiple of the XCD count (the extra ones exit at once).
static int64_t lp_grid(const GemmBatch& bt, int tiles) {
  const int64_t tm = (bt.M + LT - 1) / LT, tn = (bt.N + LT - 1) / LT;
  const int64_t bm = (tm + 3) / 4, bn = (tn + 3) / 4;
  const int64_t nblk = tiles == kLowerTiles ? bt.nmerge * bm * (bm + 1) / 2 : bt.nmerge * bm * bn;
  return (nblk + kNumXcd - 1) / kNumXcd * kNumXcd * 16;
}

template <int F16, int NSPLIT, int AM, int BM, int TILES, int ORDER, int KLO, int KHI, int EPI>
static hipError_t go_lp(const LpGemmArgs& a, hipStream_t s, int64_t total) {
  typedef LpShape<NSPLIT, lp_kt(NSPLIT, KLO)> S;
  size_t lds = (size_t)S::NBUF * S::NT * S::TILE * sizeof(unsigned short);
  if (EPI == kLpEpResid && lds < (size_t)kEpLdsBytes) lds = kEpLdsBytes;
  auto k = k_gemm_lp<F16, NSPLIT, AM, BM, TILES, ORDER, KLO, KHI, EPI>;
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  TRINV_LAUNCH(k, dim3((unsigned)total), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int F16>
static hipError_t dispatch_lp(const LpGemmArgs& a, const LpConfig& c, hipStream_t s, int64_t total) {
  // forward level product 1: T = C * A^-1 (B = A^-1 lower, transposed storage)
  if (c.nsplit == 1 && c.amask == 0 && c.bmask == 1 && c.tiles == kAllTiles && c.order == kColAsc &&
      c.klo == kLoN0 && c.khi == kHiK && c.epi == kLpEpT)
    return go_lp<F16, 1, 0, 1, kAllTiles, kColAsc, kLoN0, kHiK, kLpEpT>(a, s, total);
  // forward level product 2: X21 = -B^-1 * T (A = B^-1 lower)
  if (c.nsplit == 1 && c.amask == 1 && c.bmask == 0 && c.tiles == kAllTiles && c.order == kRowDesc &&
      c.klo == kLoZero && c.khi == kHiM1 && c.epi == kLpEpX21)
    return go_lp<F16, 1, 1, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kLpEpX21>(a, s, total);
  // residual and correction: lower tiles, each over its own K range, on
  // panel-blocked planes (zero outside their triangles, no masks)
  if (c.amask == 0 && c.bmask == 0 && c.tiles == kLowerTiles && c.order == kDiagDesc && c.klo == kLoN0Pb &&
      c.khi == kHiM1) {
    // K = 16 per stage for 2 or 3 products, 32 for one
    if (c.epi == kLpEpResid && c.nsplit == 3)
      return go_lp<F16, 3, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpResid>(a, s, total);
    if (c.epi == kLpEpResid && c.nsplit == 2)
      return go_lp<F16, 2, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpResid>(a, s, total);
    if (c.epi == kLpEpResid && c.nsplit == 1)
      return go_lp<F16, 1, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpResid>(a, s, total);
    if (c.epi == kLpEpCorr && c.nsplit == 1)
      return go_lp<F16, 1, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpCorr>(a, s, total);
  }
  return hipErrorInvalidValue;
}

// +-2^e with |e| <= 100: exact in FP32 and far from its overflow and underflow
static bool pow2_in_f32(double v) {
  int e = 0;
  const double m = std::frexp(std::fabs(v), &e);
  return m == 0.5 && e >= -99 && e <= 101;
}

hipError_t launch_gemm_lp(const LpGemmArgs& a, const LpConfig& c, hipStream_t s) {
  if (a.bt.nbatch != 1) return hipErrorInvalidValue;
  // per-lane source offsets are 32-bit byte offsets within 256 rows of a
  // row-major plane (panel-blocked planes: within one 8 KB block)
  if (c.klo != kLoN0Pb && (a.lda < 0 || a.ldb < 0 || 2 * LT * (a.lda > a.ldb ? a.lda : a.ldb) >= (int64_t)1 << 32))
    return hipErrorInvalidValue;
  const int64_t total = lp_grid(a.bt, c.tiles);
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  if (c.tiles == kLowerTiles && a.bt.M != a.bt.N) return hipErrorInvalidValue;
  // T and X21 epilogues scale by powers of two in FP32 (exact) and multiply by
  // 1 / lp_scale in place of dividing
  if (c.epi == kLpEpT && !pow2_in_f32(a.alpha)) return hipErrorInvalidValue;
  if (c.epi == kLpEpX21 && !(pow2_in_f32(a.lp_scale) && pow2_in_f32(a.alpha * a.lp_scale)))
    return hipErrorInvalidValue;
  return c.f16 ? dispatch_lp<1>(a, c, s, total) : dispatch_lp<0>(a, c, s, total);
}

}  // namespace trinv
