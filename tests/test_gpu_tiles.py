"""The tile projections for batches (on by default; APPGA_BACK_TILES=0 or
APPGA_FWD_TILES=0 at matrix load selects the row kernels): A x and A^T r against
the oracle, and whole solves against the row kernels and the oracle."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2409_13344_amd import appga as ap  # noqa: E402
from paper_2409_13344_amd import synth  # noqa: E402

GEOMS = [synth.Geometry(64, 96, 90), synth.Geometry(128, 200, 168), synth.Geometry(37, 60, 31)]
GEOM_IDS = ["64", "128", "37"]


def say(msg):
    print("[gpu-tiles] " + msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    c = ap.appga_create(0)
    yield c
    ap.appga_destroy(c)


def load(ctx, A, geom, storage, back=True, fwd=True, split=None, part_windows=None):
    """Loads a matrix with the tile projections switched on or off (part_windows:
    windows per workgroup of the forward tiles, 0 = whole tiles)."""
    keys = ("APPGA_BACK_TILES", "APPGA_FWD_TILES", "APPGA_BACK_SPLIT", "APPGA_FWD_PART_WINDOWS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ["APPGA_BACK_TILES"] = "1" if back else "0"
    os.environ["APPGA_FWD_TILES"] = "1" if fwd else "0"
    if part_windows is not None:
        os.environ["APPGA_FWD_PART_WINDOWS"] = str(part_windows)
    else:
        os.environ.pop("APPGA_FWD_PART_WINDOWS", None)
    if split is not None:
        os.environ["APPGA_BACK_SPLIT"] = str(split)
    else:
        os.environ.pop("APPGA_BACK_SPLIT", None)
    try:
        return ap.load_matrix(ctx, A, geom, storage)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("geom", GEOMS, ids=GEOM_IDS)
@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("split", [1, 2])
def test_back_tiles_operator(ctx, geom, storage, split):
    say("A^T r, %dx%d, %s, split %d" % (geom.n, geom.n, storage, split))
    A = synth.cached_matrix(geom)
    mat = load(ctx, A, geom, storage, split=split)
    try:
        deq = ap.appga_matrix_dequantized(mat, A.nnz)
        B = 64
        r = np.random.default_rng(11).standard_normal((B, geom.m)).astype(np.float32)
        out = torch.empty((B, geom.d), dtype=torch.float32, device="cuda")
        ap.appga_op_back(ctx, mat, torch.as_tensor(r).cuda(), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    Aq = synth.SparseMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col, deq)
    absA = oracle.back(Aq, np.ones(geom.m))
    for b in (0, 29, 63):
        ref = oracle.back(Aq, r[b].astype(np.float64))
        err = np.abs(got[b] - ref).max()
        assert err <= 1e-5 * np.abs(r[b]).max() * absA.max(), (b, err)


@pytest.mark.parametrize("geom", GEOMS, ids=GEOM_IDS)
@pytest.mark.parametrize("storage", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("part_windows", [0, 3])
def test_fwd_tiles_operator(ctx, geom, storage, part_windows):
    """y = A x + gamma and e = 1 - g / max(y, tau) over the ray tiles, 64 solves
    (and 128: two chunks), whole tiles per workgroup or tiles split into runs of
    3 windows (partial sums and the reduction), against the oracle on the
    dequantised matrix."""
    A = synth.cached_matrix(geom)
    mat = load(ctx, A, geom, storage, part_windows=part_windows)
    rng = np.random.default_rng(12)
    try:
        info = ap.appga_matrix_tiles(mat, ap.APPGA_TILES_FORWARD)
        assert info["valid"] == 1
        deq = ap.appga_matrix_dequantized(mat, A.nnz)
        for B in (64, 128):
            say("A x, %dx%d, %s, B %d" % (geom.n, geom.n, storage, B))
            x = rng.uniform(0.0, 2.0, (B, geom.d)).astype(np.float32)
            gam = rng.uniform(0.0, 0.5, (B, geom.m)).astype(np.float32)
            g = rng.poisson(3.0, (B, geom.m)).astype(np.float32)
            xt, gt, gmt = (torch.as_tensor(v).cuda() for v in (x, g, gam))
            y = torch.empty((B, geom.m), dtype=torch.float32, device="cuda")
            e = torch.empty_like(y)
            ap.appga_op_forward(ctx, mat, xt, gmt, y)
            ap.appga_op_ratio(ctx, mat, xt, gt, gmt, e)
            torch.cuda.synchronize()
            yg, eg = y.cpu().numpy(), e.cpu().numpy()
            Aq = synth.SparseMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col, deq)
            absx = oracle.forward(synth.SparseMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(deq)),
                                  np.full(geom.d, 2.0))
            for b in (0, 37, B - 1):
                ref = oracle.forward(Aq, x[b].astype(np.float64)) + gam[b]
                tol = 4e-6 * (absx + gam[b]) + 1e-30
                assert np.all(np.abs(yg[b] - ref) <= tol), (b, np.abs(yg[b] - ref).max())
                yc = np.maximum(ref, np.maximum(1e-6 * gam[b], 1e-30))
                eref = 1.0 - g[b] / yc
                assert np.all(np.abs(eg[b] - eref) <= 1e-5 * (1.0 + g[b] / yc)), b
    finally:
        ap.appga_free_system_matrix(ctx, mat)


def test_split1_solve_equals_row_kernel(ctx):
    """With one workgroup per tile the back projection tiles sum each pixel's
    entries in the transpose's order, exactly like the row kernel: whole solves
    (row-kernel forward in both) agree bit for bit."""
    geom = synth.Geometry(128, 200, 168)
    pr = synth.make_problem(geom, [1000, 1001, 1002, 1003], tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
    params = [ap.make_params(lam=0.02, eps=1e-3, omega=om, iterations=60) for om in (0.3, 0.5, 0.8, 1.0)]
    res = []
    for tiles in (False, True):
        mat = load(ctx, pr.A, geom, "bf16", back=tiles, fwd=False, split=1)
        try:
            f, _ = ap.appga_reconstruct_batch(ctx, mat, geom.d, pr.g, pr.gamma, params)
        finally:
            ap.appga_free_system_matrix(ctx, mat)
        res.append(f)
    np.testing.assert_array_equal(res[0], res[1])


@pytest.mark.parametrize("fwd,split", [(False, 2), (True, 1), (True, 2)])
def test_tile_solves_match_oracle(ctx, fwd, split):
    geom = synth.Geometry(128, 200, 168)
    pr = synth.make_problem(geom, [1000, 1001, 1002, 1003], tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
    params = [ap.make_params(lam=0.02, eps=1e-3, omega=0.5, iterations=100)] * 4
    mat = load(ctx, pr.A, geom, "f32", back=True, fwd=fwd, split=split)
    try:
        f, stats = ap.appga_reconstruct_batch(ctx, mat, geom.d, pr.g, pr.gamma, params)
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    for b in (0, 3):
        run = lambda rf: oracle.appga(pr.A, 128, 168, pr.g[b], pr.gamma[b], 0.02, 0.02, 1e-3, 0.5, 100,
                                      round_f32=rf)["f"]
        ref = run(False)
        floor = rel_l2(run(True), ref)
        err = rel_l2(f[b], ref)
        tol = max(1e-5, 4.0 * floor)
        say("fwd tiles %s, back split %d: solve %d vs oracle %.3e (floor %.2e)" % (fwd, split, b, err, floor))
        assert err <= tol
        assert stats[b]["guard_clamps"] == 0
