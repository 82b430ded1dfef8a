"""GPU parity of the factored forward model A = diag(n) G H (Section 4.1's PSF,
attenuation and scatter/randoms background) against the FP64 oracle.

* Operators at 128^2 (the paper's field of view at half its resolution, PSF FWHM
  6.59 mm = 2.8 pixels): A x + gamma and A^T r against att * G (H x) and
  H G^T (att * r) formed from the oracle's pieces.  Gate: 4e-6 of the
  magnitude |A| |x| (FP32 sums of a few hundred terms).
* Whole solves (APPGA and AFPPA) at 32^2 against the oracle run on the
  explicit matrix A = diag(n) G H, floor-aware: relative L2 <= max(1e-5,
  4 x floor), the floor being how far a 1e-7 relative perturbation of the data
  moves the oracle's result.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2409_13344_amd import appga as ap  # noqa: E402
from paper_2409_13344_amd import synth  # noqa: E402


def say(msg):
    print("[gpu-factored] " + msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    c = ap.appga_create(0)
    yield c
    ap.appga_destroy(c)


def load(ctx, pp, storage="f32"):
    G, geom = pp.G, pp.geom
    return ap.appga_load_system_matrix_factored(ctx, geom.n, geom.n_angles, geom.n_bins, G.row_ptr, G.col,
                                                G.val, storage, row_factors=pp.att, psf_fwhm_px=pp.fwhm_px)


@pytest.fixture(scope="module")
def p128():
    geom = synth.Geometry(128, 200, 168)
    return synth.make_physics_problem(geom, [5, 6], tc=1e6, fov_mm=300.0,
                                      G=synth.cached_matrix(geom))


@pytest.mark.parametrize("B", [1, 64])
def test_operators_128(ctx, p128, B):
    pp = p128
    geom = pp.geom
    say("factored operators 128^2, FWHM %.2f px, B=%d" % (pp.fwhm_px, B))
    mat = load(ctx, pp)
    try:
        fw, R = ap.appga_matrix_psf(mat)
        assert abs(fw - pp.fwhm_px) < 1e-12 and R == oracle.psf_radius(pp.fwhm_px)
        rng = np.random.default_rng(B)
        x = rng.uniform(0.0, 2.0, (B, geom.d)).astype(np.float32)
        gam = rng.uniform(0.5, 1.5, (B, geom.m)).astype(np.float32)
        r = rng.standard_normal((B, geom.m)).astype(np.float32)
        x_t = torch.as_tensor(x).cuda()
        gam_t = torch.as_tensor(gam).cuda()
        r_t = torch.as_tensor(r).cuda()
        y_t = torch.empty((B, geom.m), dtype=torch.float32, device="cuda")
        b_t = torch.empty((B, geom.d), dtype=torch.float32, device="cuda")
        ap.appga_op_forward(ctx, mat, x_t, gam_t, y_t)
        ap.appga_op_back(ctx, mat, r_t, b_t)
        y, bk = y_t.cpu().numpy(), b_t.cpu().numpy()
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    absG = synth.SparseMatrix(pp.G.n_rows, pp.G.n_cols, pp.G.row_ptr, pp.G.col, np.abs(pp.G.val))
    for b in sorted({0, B // 2, B - 1}):
        xb = x[b].astype(np.float64)
        ref = pp.att * oracle.forward(pp.G, oracle.psf_apply(geom.n, pp.fwhm_px, xb)) + gam[b]
        mag = pp.att * oracle.forward(absG, oracle.psf_apply(geom.n, pp.fwhm_px, np.abs(xb))) + gam[b]
        err = np.abs(y[b] - ref) / mag
        refb = oracle.psf_apply(geom.n, pp.fwhm_px, oracle.back(pp.G, pp.att * r[b]))
        magb = oracle.psf_apply(geom.n, pp.fwhm_px, oracle.back(absG, pp.att * np.abs(r[b])))
        errb = np.abs(bk[b] - refb) / np.maximum(magb, 1e-30)
        say("  solve %d: forward max rel %.2e, back max rel %.2e" % (b, err.max(), errb.max()))
        assert err.max() <= 4e-6 and errb.max() <= 4e-6


@pytest.mark.parametrize("fwhm", [1.5, 5.5, 9.0])
def test_operators_wide_psf(ctx, fwhm):
    """Other PSF widths in the lane layout, one for each blur kernel: R = 2 (the one-launch
    2-D kernel, which takes R <= 4), R = 8 (the largest radius of the run kernel) and R = 12
    (the per-output kernel). 64 solves on a 45^2 image (tiles and runs of 8 pixels end
    ragged); forward and back operators against the oracle's pieces."""
    geom = synth.Geometry(45, 64, 60)
    pp = synth.make_physics_problem(geom, [21], tc=3e5, fov_mm=45 * 2.34, G=synth.cached_matrix(geom))
    R = oracle.psf_radius(fwhm)
    say("factored operators 45^2, FWHM %.1f px (R = %d), B = 64" % (fwhm, R))
    G = pp.G
    mat = ap.appga_load_system_matrix_factored(ctx, geom.n, geom.n_angles, geom.n_bins, G.row_ptr, G.col, G.val,
                                               "f32", row_factors=pp.att, psf_fwhm_px=fwhm)
    try:
        assert ap.appga_matrix_psf(mat)[1] == R
        rng = np.random.default_rng(int(fwhm * 10))
        B = 64
        x = rng.uniform(0.0, 2.0, (B, geom.d)).astype(np.float32)
        gam = rng.uniform(0.5, 1.5, (B, geom.m)).astype(np.float32)
        r = rng.standard_normal((B, geom.m)).astype(np.float32)
        y_t = torch.empty((B, geom.m), dtype=torch.float32, device="cuda")
        b_t = torch.empty((B, geom.d), dtype=torch.float32, device="cuda")
        ap.appga_op_forward(ctx, mat, torch.as_tensor(x).cuda(), torch.as_tensor(gam).cuda(), y_t)
        ap.appga_op_back(ctx, mat, torch.as_tensor(r).cuda(), b_t)
        y, bk = y_t.cpu().numpy(), b_t.cpu().numpy()
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    absG = synth.SparseMatrix(G.n_rows, G.n_cols, G.row_ptr, G.col, np.abs(G.val))
    for b in (0, 31, 63):
        xb = x[b].astype(np.float64)
        ref = pp.att * oracle.forward(G, oracle.psf_apply(geom.n, fwhm, xb)) + gam[b]
        mag = pp.att * oracle.forward(absG, oracle.psf_apply(geom.n, fwhm, np.abs(xb))) + gam[b]
        refb = oracle.psf_apply(geom.n, fwhm, oracle.back(G, pp.att * r[b]))
        magb = oracle.psf_apply(geom.n, fwhm, oracle.back(absG, pp.att * np.abs(r[b])))
        err = (np.abs(y[b] - ref) / mag).max()
        errb = (np.abs(bk[b] - refb) / np.maximum(magb, 1e-30)).max()
        say("  solve %d: forward max rel %.2e, back max rel %.2e" % (b, err, errb))
        assert err <= 4e-6 and errb <= 4e-6


@pytest.fixture(scope="module")
def small():
    geom = synth.Geometry(32, 48, 40)
    pp = synth.make_physics_problem(geom, [11, 12, 13], tc=3e5, fov_mm=32 * 2.34)
    A = oracle.factored_matrix(pp.G, geom.n, pp.fwhm_px, pp.att)
    return pp, A


def floor_run(fn, g, seed):
    ref = fn(g)
    pert = np.asarray(g, np.float64) * (1.0 + 1e-7 * np.random.default_rng(seed).standard_normal(g.shape))
    return ref, rel_l2(fn(pert)["f"], ref["f"])


@pytest.mark.parametrize("B", [1, 3])
def test_appga_solves_32(ctx, small, B):
    pp, A = small
    geom = pp.geom
    say("factored APPGA 32^2, B=%d" % B)
    mat = load(ctx, pp)
    try:
        params = [ap.make_params(lam=0.02, eps=1e-3, omega=0.5, iterations=60)] * B
        f, st = ap.appga_reconstruct_batch(ctx, mat, geom.d, pp.g[:B], pp.gamma[:B], params)
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    for b in range(B):
        run = lambda g: oracle.appga(A, 32, 40, g, pp.gamma[b], 0.02, 0.02, 1e-3, 0.5, 60, history=True)
        ref, floor = floor_run(run, pp.g[b].astype(np.float64), b)
        e = rel_l2(f[b], ref["f"])
        say("  solve %d: image %.2e (floor %.1e), Phi %.10e vs %.10e" % (b, e, floor, st[b]["objective"],
                                                                       ref["obj"][-1]))
        assert e <= max(1e-5, 4.0 * floor)
        assert abs(st[b]["objective"] - ref["obj"][-1]) <= 1e-7 * abs(ref["obj"][-1])
        assert abs(st[b]["objective0"] - ref["obj"][0]) <= 1e-7 * abs(ref["obj"][0])


@pytest.mark.parametrize("B", [1, 3])
def test_afppa_solves_32(ctx, small, B):
    pp, A = small
    geom = pp.geom
    say("factored AFPPA 32^2, B=%d" % B)
    mat = load(ctx, pp)
    try:
        params = [ap.make_params(lam=0.02, omega=0.5, iterations=60)] * B
        f, du, st = ap.appga_afppa_batch(ctx, mat, geom.d, pp.g[:B], pp.gamma[:B], params, duals=True)
    finally:
        ap.appga_free_system_matrix(ctx, mat)
    for b in range(B):
        run = lambda g: oracle.afppa(A, 32, 40, g, pp.gamma[b], 0.02, 0.02, 0.5, 60, history=True,
                                     duals=True)
        ref, floor = floor_run(run, pp.g[b].astype(np.float64), b)
        e = rel_l2(f[b], ref["f"])
        ey = rel_l2(du[b], np.concatenate([ref["b"], ref["c"]]))
        say("  solve %d: image %.2e (floor %.1e), duals %.2e, Phi %.10e vs %.10e" % (
            b, e, floor, ey, st[b]["objective"], ref["obj"][-1]))
        assert e <= max(1e-5, 4.0 * floor)
        assert ey <= 1e-4
        assert abs(st[b]["objective"] - ref["obj"][-1]) <= 1e-7 * abs(ref["obj"][-1])


def test_factored_errors(ctx, small):
    pp, _ = small
    geom, G = pp.geom, pp.G
    bad = pp.att.copy()
    bad[3] = -1.0
    with pytest.raises(ap.AppgaError, match="row factor"):
        ap.appga_load_system_matrix_factored(ctx, geom.n, geom.n_angles, geom.n_bins, G.row_ptr, G.col, G.val,
                                             row_factors=bad)
    with pytest.raises(ap.AppgaError, match="psf_fwhm_px"):
        ap.appga_load_system_matrix_factored(ctx, geom.n, geom.n_angles, geom.n_bins, G.row_ptr, G.col, G.val,
                                             psf_fwhm_px=30.0)
    mat = load(ctx, pp)
    try:
        srv = ap.appga_server_start(ctx, 1 << 30, 64)
        try:
            with pytest.raises(ap.AppgaError, match="PSF"):
                ap.appga_submit(srv, mat, pp.g[0], pp.gamma[0], ap.make_params(lam=0.02, iterations=5))
        finally:
            ap.appga_server_stop(srv)
        d_t = torch.zeros((1, geom.d), dtype=torch.float32, device="cuda")
        with pytest.raises(ap.AppgaError, match="does not model a PSF"):
            ap.appga_op_step(ctx, mat, torch.zeros((1, geom.m), dtype=torch.float32, device="cuda"), None,
                             [0.02], [0.02], [1e-3], [1.0], [0.0], d_t, d_t.clone(), d_t.clone())
    finally:
        ap.appga_free_system_matrix(ctx, mat)
