"""Pins of the FP64 oracle of FPPA, AFPPA-N and AFPPA-GN on the nonsmooth HOITV
model (Section 4.3) against what the mathematics fixes.

- Nesterov's sequence is pinned by its defining identity.
- The HOITV value is pinned by group norms built with numpy.kron and by the
  Huber limit of the smoothed regulariser.
- The iteration is pinned by:
  - the KKT conditions of the nonsmooth model at its limit;
  - an objective no random perturbation improves on;
  - the reduction to MLEM and to APPGA when lambda = 0;
  - equivariance under scaling of the data;
  - dual feasibility;
  - the averaged-operator property of FPPA in the Condat-Vu metric.
"""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

import oracle
from paper_2409_13344_amd import synth


def dense_D(n):
    """Backward differences of Section 2.1: row 0 zero, rows j >= 1 hold +1 at j, -1 at j-1."""
    D = np.zeros((n, n))
    for j in range(1, n):
        D[j, j] = 1.0
        D[j, j - 1] = -1.0
    return D


def dense_B(n):
    D = dense_D(n)
    I = np.eye(n)
    B1 = np.vstack([np.kron(I, D), np.kron(D, I)])
    B2 = np.vstack([np.kron(I, -D.T @ D), np.kron(-D.T, D), np.kron(-D.T @ D, I),
                    np.kron(D, -D.T)])
    return B1, B2


def csr(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))


def hoitv_numpy(n, l1, l2, f):
    B1, B2 = dense_B(n)
    u = (B1 @ f).reshape(2, -1)
    v = (B2 @ f).reshape(4, -1)
    return l1 * np.linalg.norm(u, axis=0).sum() + l2 * np.linalg.norm(v, axis=0).sum()


def phi_numpy(S, n, g, gam, l1, l2, f):
    """Fidelity <Ax, 1> - <ln(Ax + gamma), g> plus HOITV (model HOTV)."""
    ax = S @ f
    return ax.sum() - g @ np.log(ax + gam) + hoitv_numpy(n, l1, l2, f)


class Problem:
    pass


@pytest.fixture(scope="module")
def prob():
    P = Problem()
    geom = synth.Geometry(8, 12, 16)
    pr = synth.make_problem(geom, [21], tc=2e4, rf=0.1)
    P.n, P.na = 8, 16
    P.A = pr.A
    P.S = csr(pr.A)
    P.g = pr.g[0].astype(np.float64)
    P.gam = pr.gamma[0].astype(np.float64)
    P.f_true = pr.f_true[0].astype(np.float64)
    P.f1 = np.full(64, P.f_true.mean())
    P.lam_col = np.asarray(P.S.sum(axis=0)).ravel()
    # Lipschitz constant of grad F on f >= 0: ||A||^2 max g / gamma^2
    P.L = np.linalg.norm(P.S.toarray(), 2) ** 2 * np.max(P.g / P.gam ** 2)
    P.lam = 0.3
    return P


@pytest.fixture(scope="module")
def long_gn(prob):
    """AFPPA-GN (omega = 1/2) with a fixed scalar P = 0.5 / L, run to its limit."""
    P = prob
    p = 0.5 / P.L
    r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, 0.5, 30000,
                     momentum=oracle.MOMENTUM_GN, precond=oracle.PRECOND_FIXED, fixed_p_scalar=p,
                     f_init=P.f1, duals=True, history=True)
    return dict(p=p, r=r)


# --------------------------------------------------------- Nesterov's sequence ---

def test_nesterov_sequence():
    """t_0 = 1 and t_k the positive root of t^2 - t = t_{k-1}^2; then t_k >= (k + 2) / 2,
    theta_1 = 0 and theta_k = (t_{k-1} - 1) / t_k increases towards 1."""
    t = [oracle.t_nesterov(k) for k in range(200)]
    assert t[0] == 1.0
    assert abs(t[1] - (1.0 + math.sqrt(5.0)) / 2.0) < 1e-15
    for k in range(1, 200):
        assert abs(t[k] * t[k] - t[k] - t[k - 1] ** 2) <= 1e-12 * t[k] ** 2
        assert t[k] >= (k + 2) / 2.0
    th = [oracle.theta_nesterov(k) for k in range(1, 200)]
    assert th[0] == 0.0
    assert all(b > a for a, b in zip(th, th[1:]))
    assert th[-1] < 1.0 and th[-1] > 0.98


# ------------------------------------------------------------------ HOITV value ---

@pytest.mark.parametrize("n", [2, 3, 8])
def test_hoitv_value_matches_kron_groups(n):
    """Group norms over pixel i of (B1 f) (2 components) and (B2 f) (4 components)."""
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n * n)
    for l1, l2 in ((1.0, 0.0), (0.0, 1.0), (0.3, 0.7)):
        assert abs(oracle.hoitv_value(n, l1, l2, f) - hoitv_numpy(n, l1, l2, f)) <= 1e-12 * (
            1.0 + hoitv_numpy(n, l1, l2, f))
    assert oracle.hoitv_value(n, 0.5, 0.5, np.full(n * n, 3.7)) == 0.0
    assert abs(oracle.hoitv_value(n, 0.5, 0.5, -2.5 * f) - 2.5 * oracle.hoitv_value(n, 0.5, 0.5, f)) \
        <= 1e-12 * oracle.hoitv_value(n, 0.5, 0.5, f)


def test_hoitv_is_the_huber_limit():
    """The smoothed regulariser is the Huber envelope of each group norm, so
    0 <= HOITV - SHOITV_eps <= (lambda1 + lambda2) d eps / 2, and the gap closes as eps -> 0."""
    n, l1, l2 = 8, 0.4, 0.2
    f = np.random.default_rng(1).uniform(0.0, 3.0, n * n)
    h = oracle.hoitv_value(n, l1, l2, f)
    for eps in (1e-1, 1e-3, 1e-6):
        gap = h - oracle.reg_value(n, l1, l2, eps, f)
        assert -1e-12 * h <= gap <= (l1 + l2) * n * n * eps / 2.0 * (1 + 1e-12)


def test_objective_hoitv_pieces(prob):
    P = prob
    f = np.random.default_rng(2).uniform(0.0, 50.0, 64)
    val = oracle.objective_hoitv(P.A, P.n, P.g, P.gam, 0.3, 0.2, f)
    assert abs(val - phi_numpy(P.S, P.n, P.g, P.gam, 0.3, 0.2, f)) <= 1e-11 * abs(val)
    assert abs(val - oracle.hoitv_value(P.n, 0.3, 0.2, f)
               - oracle.objective(P.A, P.n, P.g, P.gam, 0.0, 0.0, 1.0, f)) <= 1e-11 * abs(val)


# -------------------------------------------------------- reductions, lambda = 0 ---

def test_lambda_zero_first_step_is_mlem(prob):
    """With lambda = 0, no momentum, beta = 1 and the EM preconditioner, one step is the
    MLEM update f * A^T(g / (A f + gamma)) / Lambda, and the duals stay zero."""
    P = prob
    f0 = np.random.default_rng(3).uniform(1.0, 40.0, 64)
    r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, 0.0, 0.0, 1.0, 1, a=0.125,
                     momentum=oracle.MOMENTUM_NONE, f_init=f0, duals=True)
    mlem = f0 * (P.S.T @ (P.g / (P.S @ f0 + P.gam))) / P.lam_col
    assert np.allclose(r["f"], mlem, rtol=1e-13, atol=0)
    r5 = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, 0.0, 0.0, 0.5, 5, momentum=oracle.MOMENTUM_GN,
                      f_init=f0, duals=True)
    assert np.all(r5["b"] == 0.0) and np.all(r5["c"] == 0.0)


@pytest.mark.parametrize("momentum,omega", [(oracle.MOMENTUM_NONE, 1.0), (oracle.MOMENTUM_GN, 0.5),
                                            (oracle.MOMENTUM_GN, 1.0)])
def test_lambda_zero_matches_appga(prob, momentum, omega):
    """Without regularisation both methods are the momentum EM-preconditioned projected
    gradient step on the fidelity, whatever the smoothing parameter of APPGA."""
    P = prob
    a = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, 0.0, 0.0, omega, 25, momentum=momentum, beta=0.9,
                     history=True)
    b = oracle.appga(P.A, P.n, P.na, P.g, P.gam, 0.0, 0.0, 0.7, omega, 25, momentum=momentum, beta=0.9,
                     history=True)
    assert np.allclose(a["f"], b["f"], rtol=1e-12, atol=1e-12 * np.abs(b["f"]).max())
    assert np.allclose(a["obj"], b["obj"], rtol=1e-12, atol=0)


# ------------------------------------------------------ duals and step sizes ---

def test_dual_feasibility_and_saturation(prob):
    """b = rho (I - prox)(.) is the projection onto the lambda ball (Moreau), so every
    group has ||b_i|| <= lambda1 and ||c_i|| <= lambda2, with equality where it saturates."""
    P = prob
    for K in (1, 4, 60):
        r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, 0.5 * P.lam, 0.5, K, duals=True)
        nb = np.linalg.norm(r["b"].reshape(2, -1), axis=0)
        nc = np.linalg.norm(r["c"].reshape(4, -1), axis=0)
        assert nb.max() <= P.lam * (1 + 1e-12)
        assert nc.max() <= 0.5 * P.lam * (1 + 1e-12)
    assert nb.max() >= P.lam * (1 - 1e-12)
    assert nc.max() >= 0.5 * P.lam * (1 - 1e-12)


def test_rho_follows_the_preconditioner(prob):
    """rho1 = 1 / (2 * 8 * p_max) and rho2 = 1 / (2 * 64 * p_max), with p_max the largest
    entry of P = beta f^k / Lambda at the current (not the extrapolated) iterate."""
    P = prob
    beta = 0.8
    r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, 1.0, 3, beta=beta, history=True)
    fk = [oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, 1.0, k, beta=beta)["f"] for k in (0, 1, 2)]
    for k in range(3):
        pmax = beta * np.max(fk[k] / P.lam_col)
        assert abs(r["rho"][k, 0] - 1.0 / (16.0 * pmax)) <= 1e-13 * r["rho"][k, 0]
        assert abs(r["rho"][k, 1] - 1.0 / (128.0 * pmax)) <= 1e-13 * r["rho"][k, 1]
    rf = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, 1.0, 2, precond=oracle.PRECOND_FIXED,
                      fixed_p_scalar=0.01, history=True)
    assert np.allclose(rf["rho"], [[1 / 0.16, 1 / 1.28]] * 2, rtol=1e-14)


@pytest.mark.parametrize("momentum", [oracle.MOMENTUM_GN, oracle.MOMENTUM_NESTEROV])
def test_scaling_equivariance(prob, momentum):
    """Scaling g, gamma and f^1 by s scales every f^k by s and leaves b^k, c^k unchanged:
    grad F is invariant, P and the ball radius lambda / rho scale by s, HOITV is
    1-homogeneous.  A power-of-two s makes every rounding scale too (bit-exact)."""
    P = prob
    args = (P.lam, 0.6 * P.lam, 0.5, 40)
    r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, *args, momentum=momentum, duals=True)
    f1 = oracle.init_image(P.n, P.na, P.g, P.gam)
    r4 = oracle.afppa(P.A, P.n, P.na, 4.0 * P.g, 4.0 * P.gam, *args, momentum=momentum,
                      f_init=4.0 * f1, duals=True)
    assert np.array_equal(r4["f"], 4.0 * r["f"])
    assert np.array_equal(r4["b"], r["b"]) and np.array_equal(r4["c"], r["c"])
    r3 = oracle.afppa(P.A, P.n, P.na, 3.0 * P.g, 3.0 * P.gam, *args, momentum=momentum,
                      f_init=3.0 * f1, duals=True)
    assert np.allclose(r3["f"], 3.0 * r["f"], rtol=1e-9, atol=1e-9 * r["f"].max())
    assert np.allclose(r3["b"], r["b"], rtol=0, atol=1e-9 * P.lam)


# ------------------------------------------------------- the limit is optimal ---

@pytest.mark.slow
def test_kkt_of_the_nonsmooth_model(prob, long_gn):
    """At the limit: f >= 0; grad F(f) + B1^T b + B2^T c vanishes where f > 0 and is >= 0
    where f = 0; b_i = lambda1 (B1 f)_i / ||(B1 f)_i|| where that group is nonzero and
    ||b_i|| <= lambda1 where it is zero; c likewise with B2."""
    P, r = prob, long_gn["r"]
    f, b, c = r["f"], r["b"].reshape(2, -1), r["c"].reshape(4, -1)
    B1, B2 = dense_B(P.n)
    grad = P.S.T @ (1.0 - P.g / (P.S @ f + P.gam)) + B1.T @ b.ravel() + B2.T @ c.ravel()
    scale = np.abs(P.S.T @ (1.0 - P.g / (P.S @ P.f1 + P.gam))).max()
    assert f.min() >= 0.0
    act = f > 1e-9 * f.max()
    assert 0 < act.sum() < 64
    assert np.abs(grad[act]).max() <= 1e-9 * scale
    assert grad[~act].min() >= -1e-9 * scale
    u = (B1 @ f).reshape(2, -1)
    v = (B2 @ f).reshape(4, -1)
    for dual, w, lam in ((b, u, P.lam), (c, v, P.lam)):
        nw = np.linalg.norm(w, axis=0)
        live = nw > 1e-7 * nw.max()
        assert 0 < live.sum() < live.size
        assert np.abs(dual[:, live] - lam * w[:, live] / nw[live]).max() <= 1e-7 * lam
        assert np.linalg.norm(dual[:, ~live], axis=0).max() <= lam * (1 + 1e-12)


@pytest.mark.slow
def test_limit_is_not_improved_by_perturbations(prob, long_gn):
    """The oracle's objective agrees with a numpy one, and no nonnegative perturbation of
    the limit, nor an independent L-BFGS-B minimiser of a finely smoothed model, has a
    lower nonsmooth objective."""
    P, r = prob, long_gn["r"]
    f = r["f"]
    phi = phi_numpy(P.S, P.n, P.g, P.gam, P.lam, P.lam, f)
    assert abs(r["obj"][-1] - phi) <= 1e-11 * abs(phi)
    rng = np.random.default_rng(4)
    scale = 1e-3 * f.mean()
    for _ in range(200):
        x = np.maximum(f + scale * rng.standard_normal(64), 0.0)
        assert phi_numpy(P.S, P.n, P.g, P.gam, P.lam, P.lam, x) >= phi - 1e-12 * abs(phi)
    for j in range(64):
        for s in (+1.0, -1.0):
            x = f.copy()
            x[j] = max(x[j] + s * scale, 0.0)
            assert phi_numpy(P.S, P.n, P.g, P.gam, P.lam, P.lam, x) >= phi - 1e-12 * abs(phi)
    B1, B2 = dense_B(P.n)
    eps = 1e-4

    def smooth(x):
        y = P.S @ x + P.gam
        u = (B1 @ x).reshape(2, -1)
        v = (B2 @ x).reshape(4, -1)
        nu, nv = np.linalg.norm(u, axis=0), np.linalg.norm(v, axis=0)
        hu = np.where(nu > eps, nu - eps / 2, nu * nu / (2 * eps))
        hv = np.where(nv > eps, nv - eps / 2, nv * nv / (2 * eps))
        grad = (P.S.T @ (1 - P.g / y) + B1.T @ (P.lam * u / np.maximum(nu, eps)).ravel()
                + B2.T @ (P.lam * v / np.maximum(nv, eps)).ravel())
        return y.sum() - P.gam.sum() - P.g @ np.log(y) + P.lam * (hu.sum() + hv.sum()), grad

    best = scipy.optimize.minimize(smooth, P.f1, jac=True, method="L-BFGS-B", bounds=[(0, None)] * 64,
                                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-11, maxcor=30))
    phi_best = phi_numpy(P.S, P.n, P.g, P.gam, P.lam, P.lam, best.x)
    assert phi <= phi_best + 1e-12 * abs(phi)
    # the smoothed optimum lies within the Huber gap of the nonsmooth one
    assert phi_best - phi <= 2 * P.lam * 64 * eps


@pytest.mark.slow
@pytest.mark.parametrize("momentum,omega,K", [(oracle.MOMENTUM_GN, 0.25, 160000),
                                              (oracle.MOMENTUM_GN, 0.75, 10000),
                                              (oracle.MOMENTUM_NONE, 1.0, 400000)])
def test_every_momentum_reaches_the_same_minimiser(prob, long_gn, momentum, omega, K):
    """The model has one minimiser; FPPA and AFPPA-GN with omega < 1 reach it from the
    same start (the smaller omega, the more iterations)."""
    P = prob
    r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, omega, K, momentum=momentum,
                     precond=oracle.PRECOND_FIXED, fixed_p_scalar=long_gn["p"], f_init=P.f1)
    f = long_gn["r"]["f"]
    assert np.linalg.norm(r["f"] - f) <= 1e-6 * np.linalg.norm(f)


# ------------------------------------------------- FPPA is an averaged operator ---

def metric_norm(dz, n, p, rho1, rho2):
    """||z||_V for V = [[P^-1, -B^T], [-B, R^-1]], z = (f, b, c), B = [B1; B2],
    R = diag(rho1 I, rho2 I): the metric in which FPPA is a forward-backward step."""
    B1, B2 = dense_B(n)
    d = n * n
    f, b, c = dz[:d], dz[d:3 * d], dz[3 * d:]
    q = f @ f / p - 2.0 * b @ (B1 @ f) - 2.0 * c @ (B2 @ f) + b @ b / rho1 + c @ c / rho2
    return math.sqrt(max(q, 0.0))


def test_fppa_is_averaged_in_the_condat_vu_metric(prob):
    """Without momentum the iteration with a scalar P is forward-backward in the metric V.
    When P^-1 - B^T R B > L/2 (checked here), the map is averaged there, so both the step
    ||z^{k+1} - z^k||_V and the distance between two runs from different starts never grow."""
    P = prob
    p = 0.1 / P.L
    rho1, rho2 = 1.0 / (16.0 * p), 1.0 / (128.0 * p)
    B1, B2 = dense_B(P.n)
    M = np.eye(64) / p - rho1 * B1.T @ B1 - rho2 * B2.T @ B2
    assert np.linalg.eigvalsh(M).min() > P.L / 2.0
    starts = (P.f1, np.random.default_rng(5).uniform(0.0, 2.0 * P.f1[0], 64))
    runs = []
    for f0 in starts:
        zs = []
        for k in range(0, 31):
            r = oracle.afppa(P.A, P.n, P.na, P.g, P.gam, P.lam, P.lam, 1.0, k,
                             momentum=oracle.MOMENTUM_NONE, precond=oracle.PRECOND_FIXED,
                             fixed_p_scalar=p, f_init=f0, duals=True)
            zs.append(np.concatenate([r["f"], r["b"], r["c"]]))
        runs.append(zs)
        steps = [metric_norm(zs[k + 1] - zs[k], P.n, p, rho1, rho2) for k in range(30)]
        assert all(s1 <= s0 * (1 + 1e-9) for s0, s1 in zip(steps, steps[1:]))
        assert steps[-1] < steps[0]
    dist = [metric_norm(a - b, P.n, p, rho1, rho2) for a, b in zip(*runs)]
    assert all(d1 <= d0 * (1 + 1e-9) for d0, d1 in zip(dist, dist[1:]))


def test_afppa_rejects_bad_arguments(prob):
    P = prob
    base = dict(A=P.A, n=P.n, n_angles=P.na, g=P.g, gamma=P.gam, lam1=0.1, lam2=0.1, omega=0.5,
                iterations=2)
    for bad in (dict(omega=0.0), dict(omega=1.5), dict(lam1=-1.0), dict(beta=0.0),
                dict(precond=oracle.PRECOND_FIXED, fixed_p_scalar=0.0), dict(omega=1.0, a=0.5)):
        with pytest.raises(RuntimeError):
            oracle.afppa(**dict(base, **bad))


def test_round_f32_diagnostic():
    """The FP32-rounding diagnostic changes nothing where every held value is an FP32
    number (A = I, integer counts, lambda = 0, no momentum: each iterate is g exactly and
    the duals stay 0), and moves a real problem by an FP32-size amount."""
    n = 4
    d = n * n
    A = synth.SparseMatrix(d, d, np.arange(d + 1, dtype=np.int64), np.arange(d, dtype=np.int32), np.ones(d))
    g = np.random.default_rng(12).integers(1, 50, d).astype(np.float64)
    kw = dict(momentum=oracle.MOMENTUM_NONE, f_init=np.full(d, 2.0), duals=True)
    exact = oracle.afppa(A, n, 1, g, np.zeros(d), 0.0, 0.0, 1.0, 5, **kw)
    rounded = oracle.afppa(A, n, 1, g, np.zeros(d), 0.0, 0.0, 1.0, 5, round_f32=True, **kw)
    np.testing.assert_array_equal(exact["f"], rounded["f"])
    np.testing.assert_array_equal(exact["f"], g)
    pr = synth.config_problem("c1_64")
    args = (pr.A, 64, 90, pr.g[0], pr.gamma[0], 0.05, 0.05, 0.5, 10)
    f0 = oracle.afppa(*args, duals=True)
    f1 = oracle.afppa(*args, duals=True, round_f32=True)
    gap = np.linalg.norm(f1["f"] - f0["f"]) / np.linalg.norm(f0["f"])
    assert 1e-9 < gap < 1e-5
    assert np.abs(f1["f"] - f1["f"].astype(np.float32)).max() == 0.0
    assert np.abs(f1["b"] - f1["b"].astype(np.float32)).max() == 0.0
