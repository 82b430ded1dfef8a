"""The tile back projection for batches (opt-in with APPGA_BACK_TILES=1 at matrix
load): A^T r against the oracle, and whole solves against the row kernel and
the oracle."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2409_13344_amd import appga as ap  # noqa: E402
from paper_2409_13344_amd import synth  # noqa: E402


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


def load(ctx, A, geom, storage, tiles, split=None):
    """Loads a matrix with the tile back projection switched on or off."""
    saved = {k: os.environ.get(k) for k in ("APPGA_BACK_TILES", "APPGA_BACK_SPLIT")}
    os.environ["APPGA_BACK_TILES"] = "1" if tiles else "0"
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


@pytest.mark.parametrize("geom", [synth.Geometry(64, 96, 90), synth.Geometry(128, 200, 168),
                                  synth.Geometry(37, 60, 31)], ids=["64", "128", "37"])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("split", [1, 2])
def test_back_tiles_operator(ctx, geom, storage, split):
    say("A^T r, %dx%d, %s, split %d" % (geom.n, geom.n, storage, split))
    A = synth.cached_matrix(geom)
    mat = load(ctx, A, geom, storage, True, split)
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


def test_split1_solve_equals_row_kernel(ctx):
    """With one workgroup per tile the tile kernel sums each pixel's entries in
    the transpose's order, exactly like the row kernel: whole solves agree bit
    for bit."""
    geom = synth.Geometry(128, 200, 168)
    pr = synth.make_problem(geom, [1000, 1001, 1002, 1003], tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
    params = [ap.make_params(lam=0.02, eps=1e-3, omega=om, iterations=60) for om in (0.3, 0.5, 0.8, 1.0)]
    res = []
    for tiles in (False, True):
        mat = load(ctx, pr.A, geom, "bf16", tiles, 1)
        try:
            f, _ = ap.appga_reconstruct_batch(ctx, mat, geom.d, pr.g, pr.gamma, params)
        finally:
            ap.appga_free_system_matrix(ctx, mat)
        res.append(f)
    np.testing.assert_array_equal(res[0], res[1])


def test_split2_solve_matches_oracle(ctx):
    geom = synth.Geometry(128, 200, 168)
    pr = synth.make_problem(geom, [1000, 1001, 1002, 1003], tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
    params = [ap.make_params(lam=0.02, eps=1e-3, omega=0.5, iterations=100)] * 4
    mat = load(ctx, pr.A, geom, "f32", True, 2)
    try:
        f, stats = ap.appga_reconstruct_batch(ctx, mat, geom.d, pr.g, pr.gamma, params)
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    for b in (0, 3):
        ref = oracle.appga(pr.A, 128, 168, pr.g[b], pr.gamma[b], 0.02, 0.02, 1e-3, 0.5, 100)["f"]
        err = rel_l2(f[b], ref)
        say("split 2 solve %d vs oracle %.3e" % (b, err))
        assert err <= 1e-5
        assert stats[b]["guard_clamps"] == 0
