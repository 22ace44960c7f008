"""GPU parity of the batched inverse through the C ABI: uneven orders in one
persistent launch (FP32 and FP64), per-matrix status, unit diagonals, graph
capture and replay, and the 4096-matrix configuration.

Tolerances: FP32 relative residual ||L X - I||_F / (||L||_F ||X||_F) <= 1e-5
per matrix and relative forward error against the oracle <= 1e-4 (kappa ~ 2
for this generator, FP32 unit roundoff 6e-8 times the depth of the
recursion); FP64 residual <= 1e-13 and forward error <= 1e-11.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner

pytestmark = pytest.mark.gpu

TOL = {"f32": (1e-5, 1e-4), "f64": (1e-13, 1e-11)}


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07611_amd as P

    P.load()
    return P


def make_batch(sizes, dtype, seed0=1000, unit=False):
    offs = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        offs[1:] = np.cumsum(np.asarray(sizes[:-1], dtype=np.int64) ** 2)
    total = int(offs[-1] + int(sizes[-1]) ** 2)
    packed = np.zeros(total, dtype=dtype)
    mats = []
    for i, n in enumerate(sizes):
        L = synth.lower_triangular(int(n), seed0 + i, unit=unit, dtype=dtype)
        packed[offs[i]:offs[i] + n * n] = L.ravel()
        mats.append(L)
    return packed, offs, mats


def unpack(X, offs, sizes):
    return [X[o:o + n * n].reshape(n, n) for o, n in zip(offs, sizes)]


def rel_residual(L, X):
    L = L.astype(np.float64)
    X = X.astype(np.float64)
    n = L.shape[0]
    return np.linalg.norm(L @ X - np.eye(n)) / (np.linalg.norm(L) * np.linalg.norm(X))


def check(mats, Xs, tol, oracle_every=1, unit=False):
    rt, ft = tol
    worst_r = worst_f = 0.0
    for i, (L, X) in enumerate(zip(mats, Xs)):
        assert np.all(np.triu(X, 1) == 0), f"matrix {i}: nonzero above the diagonal"
        r = rel_residual(np.tril(L) if not unit else np.tril(L, -1) + np.eye(L.shape[0]), X)
        worst_r = max(worst_r, r)
        assert r <= rt, f"matrix {i} n={L.shape[0]}: residual {r:.3e}"
        if i % oracle_every == 0:
            Xo = oracle.tril_inverse(L.astype(np.float64), unit=unit)
            f = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
            worst_f = max(worst_f, f)
            assert f <= ft, f"matrix {i} n={L.shape[0]}: forward error {f:.3e}"
    return worst_r, worst_f


EDGE_SIZES = [1, 2, 3, 15, 16, 17, 31, 32, 33, 47, 63, 64, 65, 96, 127, 128, 129, 200, 255, 256, 257, 263, 300,
              383, 511, 512, 513, 700, 1000, 1023, 1024, 5, 64, 100]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("leaf", [0, 32, 64])
def test_uneven_batch_vs_oracle(P, dt, leaf):
    import torch

    banner(f"batched uneven {dt} leaf={leaf} sizes={len(EDGE_SIZES)}")
    npdt = np.float32 if dt == "f32" else np.float64
    packed, offs, mats = make_batch(EDGE_SIZES, npdt)
    X, st = P.tril_inverse_batched(torch.from_numpy(packed).cuda(), EDGE_SIZES, offs, dt, leaf=leaf)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    Xs = unpack(X.cpu().numpy(), offs, EDGE_SIZES)
    r, f = check(mats, Xs, TOL[dt])
    print(f"{dt} leaf={leaf}: worst residual {r:.3e}, worst forward error {f:.3e}", flush=True)


def test_uneven_batch_singular_and_offsets(P):
    """Per-matrix status (1-based first zero pivot) and non-contiguous offsets
    (gaps between the matrices are left untouched)."""
    import torch

    banner("batched singular + gaps")
    sizes = [40, 300, 7, 129, 64]
    gap = 37
    offs = np.zeros(len(sizes), dtype=np.int64)
    for i in range(1, len(sizes)):
        offs[i] = offs[i - 1] + sizes[i - 1] ** 2 + gap
    total = int(offs[-1] + sizes[-1] ** 2)
    packed = np.full(total, -7.0, dtype=np.float32)
    mats = []
    for i, n in enumerate(sizes):
        L = synth.lower_triangular(n, 50 + i, dtype=np.float32)
        mats.append(L)
        packed[offs[i]:offs[i] + n * n] = L.ravel()
    packed[offs[1] + 150 * 300 + 150] = 0.0  # matrix 1: L[150, 150] = 0
    packed[offs[3] + 0] = 0.0  # matrix 3: L[0, 0] = 0
    Xd = torch.full((total,), 3.5, dtype=torch.float32, device="cuda")
    _, st = P.tril_inverse_batched(torch.from_numpy(packed).cuda(), sizes, offs, "f32", out=Xd)
    torch.cuda.synchronize()
    assert st.cpu().numpy().tolist() == [0, 151, 0, 1, 0]
    X = Xd.cpu().numpy()
    for i in range(1, len(sizes)):  # gaps untouched
        assert np.all(X[offs[i] - gap:offs[i]] == 3.5)
    Xs = unpack(X, offs, sizes)
    for i in (0, 2, 4):
        assert rel_residual(mats[i], Xs[i]) <= 1e-5


def test_uneven_batch_unit_diagonal(P):
    import torch

    banner("batched unit diagonal")
    sizes = [33, 260, 1, 90, 512]
    packed, offs, mats = make_batch(sizes, np.float64, seed0=70)
    lib = P._lib
    # unit flag through the C ABI directly (the Python wrapper has no unit option here)
    import ctypes

    L_d = torch.from_numpy(packed).cuda()
    Xu = torch.empty_like(L_d)
    stu = torch.empty(len(sizes), dtype=torch.int32, device="cuda")
    n_np = np.asarray(sizes, dtype=np.int32)
    n_d = torch.from_numpy(n_np).cuda()
    o_d = torch.from_numpy(offs).cuda()
    o = lib.Opts()
    lib.load().trinv_default_opts(ctypes.byref(o))
    o.unit_diag = 1
    o.blocking = 1
    nb = lib.load().trinv_batched_workspace_bytes(lib.F64, len(sizes), n_np.ctypes.data, ctypes.byref(o))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    rc = lib.load().trinv_tril_inverse_batched(lib.F64, len(sizes), n_np.ctypes.data, n_d.data_ptr(),
                                                offs.ctypes.data, o_d.data_ptr(), L_d.data_ptr(), Xu.data_ptr(),
                                                stu.data_ptr(), ctypes.byref(o), ws.data_ptr(), nb,
                                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0 and np.all(stu.cpu().numpy() == 0)
    check(mats, unpack(Xu.cpu().numpy(), offs, sizes), TOL["f64"], unit=True)


def test_graph_replay_matches_eager(P):
    """Capture once, replay with new inputs written into the static buffer and
    eager work in between; every replay equals the eager call bit for bit
    (each matrix's arithmetic does not depend on which workgroup runs it)."""
    import torch

    banner("batched graph capture/replay")
    sizes = synth.batch_sizes(300, seed=11)
    g = P.BatchedGraph(sizes, dtype=torch.float32)
    g.capture()
    for rep, seed0 in enumerate([1000, 5000, 9000]):
        packed, offs, mats = make_batch(sizes, np.float32, seed0=seed0)
        g.L.copy_(torch.from_numpy(packed).cuda())
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        Xg = g.X.clone()
        stg = g.status.clone()
        Xe, ste = P.tril_inverse_batched(g.L, sizes, offs, "f32")
        torch.cuda.synchronize()
        assert torch.equal(Xg, Xe), f"replay {rep} differs from eager"
        assert torch.equal(stg, ste)
        if rep == 0:
            check(mats, unpack(Xg.cpu().numpy(), offs, sizes), TOL["f32"], oracle_every=10)


def test_batched_4096_configuration(P):
    """4096 FP32 matrices, n_i = 16 + (splitmix(6, i) mod 497): residual of
    every matrix in FP64 on the host, oracle comparison on every 16th."""
    import torch

    sizes = synth.batch_sizes(4096)
    banner(f"batched 4096 f32 sum n^2 = {int(np.sum(sizes.astype(np.int64) ** 2))}")
    packed, offs, mats = make_batch(sizes, np.float32)
    X, st = P.tril_inverse_batched(torch.from_numpy(packed).cuda(), sizes, offs, "f32")
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    r, f = check(mats, unpack(X.cpu().numpy(), offs, sizes), TOL["f32"], oracle_every=16)
    print(f"4096: worst residual {r:.3e}, worst forward error {f:.3e}", flush=True)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n,batch", [(300, 10), (1024, 3), (64, 40), (130, 300)])
def test_uniform_batches(P, dt, n, batch):
    """Equal orders: a few large matrices run the batched level products, many
    or small ones the persistent kernel; both against the oracle."""
    import torch

    banner(f"batched uniform {dt} n={n} batch={batch}")
    sizes = [n] * batch
    npdt = np.float32 if dt == "f32" else np.float64
    packed, offs, mats = make_batch(sizes, npdt, seed0=900)
    X, st = P.tril_inverse_batched(torch.from_numpy(packed).cuda(), sizes, offs, dt)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    check(mats, unpack(X.cpu().numpy(), offs, sizes), TOL[dt], oracle_every=max(1, batch // 8))


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("leaf,per_cu,tile", [(32, 1, 128), (64, 1, 64), (32, 2, 64), (64, 2, 128), (64, 0, 0),
                                               (32, 64, 64)])
def test_pinned_configurations_vs_oracle(P, dt, leaf, per_cu, tile):
    """Every configuration the autotuner may choose gives a correct inverse of
    every matrix: leaves of 32 or 64 (the recursion's cut-off), level tiles of
    at most 64 or 128; a workgroup count per CU above the occupancy limit runs
    at that limit."""
    import torch

    banner(f"batched {dt} pinned leaf={leaf} wgs_per_cu={per_cu} tile={tile}")
    sizes = np.array(EDGE_SIZES, dtype=np.int32)
    np_dt = np.float32 if dt == "f32" else np.float64
    packed, offs, mats = make_batch(sizes, np_dt, seed0=5000)
    P.batched_set_config(sizes, dt, leaf, per_cu, tile)
    assert P.batched_get_config(sizes, dt) == {"leaf": leaf, "wgs_per_cu": per_cu, "tile": tile or 128}
    L = torch.from_numpy(packed).cuda()
    X, status = P.tril_inverse_batched(L, sizes, offs, dt)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    check(mats, unpack(X.cpu().numpy(), offs, sizes), TOL[dt], oracle_every=3)


def test_autotune_then_graph_vs_oracle(P):
    """The autotuner times its candidates on an uneven FP32 batch, keeps one of
    them, leaves that configuration's result in X, and the captured graph that
    reuses it replays to the same inverses."""
    import torch

    sizes = synth.batch_sizes(600)
    banner(f"batched autotune, {len(sizes)} FP32 matrices")
    packed, offs, mats = make_batch(sizes, np.float32, seed0=7000)
    g = P.BatchedGraph(sizes, offs, dtype=torch.float32)
    g.L.copy_(torch.from_numpy(packed).cuda())
    cfg = g.tune()
    print(f"autotune: {cfg}", flush=True)
    assert cfg["leaf"] in (32, 64) and cfg["tile"] in (64, 128) and cfg["wgs_per_cu"] >= 1 and cfg["ms"] > 0
    check(mats, unpack(g.X.cpu().numpy(), offs, sizes), TOL["f32"], oracle_every=25)
    g.X.zero_()
    g.capture(tune=False)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert int(g.status.abs().sum()) == 0
        check(mats, unpack(g.X.cpu().numpy(), offs, sizes), TOL["f32"], oracle_every=25)


def test_autotune_f64_uneven(P):
    """The tuner on an FP64 batch: a candidate configuration, correct results."""
    import torch

    sizes = np.array([17, 300, 64, 1024, 129, 512, 5, 256] * 8, dtype=np.int32)
    banner(f"batched autotune, {len(sizes)} FP64 matrices")
    packed, offs, mats = make_batch(sizes, np.float64, seed0=9000)
    L = torch.from_numpy(packed).cuda()
    X = torch.empty_like(L)
    status = torch.empty(len(sizes), dtype=torch.int32, device="cuda")
    cfg = P.batched_autotune(L, sizes, offs, "f64", out=X, status=status)
    torch.cuda.synchronize()
    print(f"autotune: {cfg}", flush=True)
    assert cfg["leaf"] in (32, 64) and cfg["tile"] in (64, 128) and cfg["wgs_per_cu"] >= 1 and cfg["ms"] > 0
    assert int(status.abs().sum()) == 0
    check(mats, unpack(X.cpu().numpy(), offs, sizes), TOL["f64"], oracle_every=5)
    X2, st2 = P.tril_inverse_batched(L, sizes, offs, "f64")
    torch.cuda.synchronize()
    assert int(st2.abs().sum()) == 0
    check(mats, unpack(X2.cpu().numpy(), offs, sizes), TOL["f64"], oracle_every=5)


_TUNE_SCRIPT = r"""
import json, os, sys
import numpy as np
import torch
sys.path.insert(0, os.environ["TRINV_TEST_ROOT"])
import paper_2307_07611_amd as P
sizes = np.array([40, 130, 77] * 100, dtype=np.int32)
sq = sizes.astype(np.int64) ** 2
offs = np.concatenate([[0], np.cumsum(sq)[:-1]]).astype(np.int64)
rng = np.random.default_rng(1)
packed = np.zeros(int(sq.sum()), dtype=np.float32)
for n, o in zip(sizes, offs):
    A = np.tril(rng.standard_normal((n, n)) / n, -1) + 2.0 * np.eye(n)
    packed[o:o + n * n] = A.ravel()
if sys.argv[1] == "tune":
    L = torch.from_numpy(packed).cuda()
    X = torch.empty_like(L)
    st = torch.empty(len(sizes), dtype=torch.int32, device="cuda")
    P.batched_autotune(L, sizes, offs, "f32", out=X, status=st)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
else:
    torch.zeros(1, device="cuda")
print("CFG " + json.dumps([P.batched_get_config(sizes, "f32"), P.batched_get_config([33] * 500, "f32")]), flush=True)
"""


def test_tune_cache_across_processes(tmp_path):
    """TRINV_TUNE_CACHE: one process tunes and appends its result; a fresh
    process loads it without tuning, and a line written for another order
    signature is honoured; without the variable the defaults apply."""
    import json
    import os
    import subprocess
    import sys

    banner("batched tuning cache across processes")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    script = tmp_path / "tune_script.py"
    script.write_text(_TUNE_SCRIPT)

    def run(arg, with_cache=True):
        env = dict(os.environ, TRINV_TEST_ROOT=root)
        env.pop("TRINV_TUNE_CACHE", None)
        if with_cache:
            env["TRINV_TUNE_CACHE"] = str(cache)
        r = subprocess.run([sys.executable, str(script), arg], capture_output=True, text=True, env=env, timeout=240)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
        line = [ln for ln in r.stdout.splitlines() if ln.startswith("CFG ")][-1]
        return json.loads(line[4:])

    tuned, other = run("tune")
    lines = cache.read_text().split("\n")
    lines = [ln for ln in lines if ln.strip()]
    assert len(lines) == 1, lines
    f = lines[0].split()
    assert len(f) == 10 and f[0].startswith("gfx") and int(f[1]) == 1 and int(f[2]) == 300
    assert (int(f[6]), int(f[7]), int(f[8])) == (tuned["leaf"], tuned["wgs_per_cu"], tuned["tile"])
    default = {"leaf": 64, "wgs_per_cu": 0, "tile": 128}  # FP32 defaults
    assert other == default  # untuned signature
    # a line for the other signature (500 matrices of order 33), same device
    with open(cache, "a") as fh:
        fh.write(f"{f[0]} 1 500 {500 * 33} {500 * 33 * 33} 33 32 1 64 0.5\n")
    loaded, other = run("read")
    assert loaded == tuned
    assert other == {"leaf": 32, "wgs_per_cu": 1, "tile": 64}
    plain, other = run("read", with_cache=False)
    assert plain == default and other == default


@pytest.mark.parametrize("dt,sizes", [("f64", [17, 300, 64, 1024, 129, 5, 256, 33] * 3),
                                      ("f32", [40, 700, 96, 1] * 6),
                                      ("f32", [256] * 8)])  # uniform: the level path
def test_upper_batch(P, dt, sizes):
    """opts.upper on a packed batch with gaps between matrices: X_i = U_i^-1
    (upper, zeros below the diagonal); the strict lower parts of the inputs
    hold NaN and must not be read; the gaps are left untouched."""
    import torch

    dtype = np.float64 if dt == "f64" else np.float32
    sizes = np.array(sizes, dtype=np.int32)
    banner(f"batched upper, {len(sizes)} {dt} matrices")
    gap = 7
    offs = np.zeros(len(sizes), dtype=np.int64)
    for i in range(1, len(sizes)):
        offs[i] = offs[i - 1] + int(sizes[i - 1]) ** 2 + gap
    total = int(offs[-1] + int(sizes[-1]) ** 2 + gap)
    packed = np.full(total, -3.0, dtype=dtype)
    lowers = []
    for i, n in enumerate(sizes):
        L = synth.lower_triangular(int(n), 7000 + i, dtype=dtype)
        U = np.ascontiguousarray(L.T)
        U[np.tril_indices(int(n), -1)] = np.nan
        packed[offs[i]:offs[i] + n * n] = U.ravel()
        lowers.append(L)
    Lg = torch.from_numpy(packed).cuda()
    X = torch.full_like(Lg, 5.0)
    Xg, st = P.tril_inverse_batched(Lg, sizes, offs, dt, upper=True, out=X)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Xh = Xg.cpu().numpy()
    for i, n in enumerate(sizes):  # gaps untouched
        end = offs[i] + n * n
        assert np.all(Xh[end:end + gap] == 5.0)
    Xs = [x.T.copy() for x in unpack(Xh, offs, sizes)]  # lower inverses of L_i = U_i^T
    check(lowers, Xs, TOL[dt], oracle_every=3)
