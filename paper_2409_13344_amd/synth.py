"""Seeded synthetic PET workloads: Siddon system matrix, ellipse phantoms, Poisson data.

This module generates inputs only.  It contains none of the reconstruction
arithmetic (no projection of iterates, no gradients, no preconditioner, no
momentum); both the GPU library's tests and the FP64 checker draw their inputs
from here so that the two see bit-identical data.

Model inputs follow Section 2.1 (system matrix A in R+^{m x d}, background
gamma in R+^m, data g = Poisson(A f + gamma), d = N^2).  The paper's own
simulation (Section 4.1: area-integral projector of a clinical ring, PSF,
attenuation, scatter) is not reproducible here, so the stand-in is:

* geometry: N x N unit pixels centred on the origin; pixel (r, c) has centre
  x = c - (N-1)/2, y = r - (N-1)/2 and index j = r*N + c (row-major);
* parallel-beam rays, angles phi_a = a*pi/A (a = 0..A-1, 180 degrees), bins
  s_b = (b - (R-1)/2)*ds; ray i = a*R + b is the line x cos(phi) + y sin(phi) = s;
* A_ij = length of ray i inside pixel j (Siddon, Med. Phys. 12(2), 1985),
  computed in FP64; rays that miss the square give empty rows;
* phantom: random ellipses inside the field-of-view disk of radius N/2;
* counts: total expected counts TC = sum(A f_true + gamma), a fraction r of
  them uniform background (the TC and RF definitions of Section 4.1).

make_physics_problem adds the physics of Section 4.1's simulation on the same
geometry: a space-invariant Gaussian PSF, uniform water attenuation, scatter
and randoms (see its docstring).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "Geometry", "SparseMatrix", "Problem", "siddon_matrix", "ellipse_phantom", "disc_phantom",
    "make_problem", "config_problem", "CONFIGS", "chord_length_square", "PhysicsProblem",
    "water_disc_mu", "make_physics_problem",
]


@dataclasses.dataclass(frozen=True)
class Geometry:
    n: int          # image side N (d = N*N)
    n_bins: int     # radial bins R
    n_angles: int   # projection angles A over 180 degrees (NPA)
    ds: float = 1.0

    @property
    def d(self) -> int:
        return self.n * self.n

    @property
    def m(self) -> int:
        return self.n_bins * self.n_angles


@dataclasses.dataclass
class SparseMatrix:
    """CSR matrix with FP64 values (the master copy shared by every consumer)."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray   # int64, n_rows + 1
    col: np.ndarray       # int32, nnz
    val: np.ndarray       # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


@dataclasses.dataclass
class Problem:
    geom: Geometry
    A: SparseMatrix
    g: np.ndarray        # (B, m) float32 counts (exact integers)
    gamma: np.ndarray    # (B, m) float32 background, uniform per sinogram
    f_true: np.ndarray   # (B, d) float64 ground truth
    tc: np.ndarray       # (B,) total expected counts
    rf: np.ndarray       # (B,) background fraction
    seeds: List[int]


def _slab(p0: np.ndarray, u: float, half: float):
    """Parameter interval where p0 + t*u lies in [-half, half] (per ray)."""
    if abs(u) < 1e-12:
        inside = np.abs(p0) < half
        lo = np.where(inside, -np.inf, np.inf)
        hi = np.where(inside, np.inf, -np.inf)
        return lo, hi
    t1 = (-half - p0) / u
    t2 = (half - p0) / u
    return np.minimum(t1, t2), np.maximum(t1, t2)


def siddon_matrix(geom: Geometry, min_seg: float = 1e-9) -> SparseMatrix:
    """FP64 line-length system matrix, CSR, rows ordered i = angle*R + bin.

    Within a row the entries follow the ray from its entry to its exit point.
    Segments shorter than ``min_seg`` (grazing a grid corner) are dropped.
    """
    n, R, A = geom.n, geom.n_bins, geom.n_angles
    half = n / 2.0
    edges = np.arange(n + 1, dtype=np.float64) - half
    sb = (np.arange(R, dtype=np.float64) - (R - 1) / 2.0) * geom.ds
    counts = np.zeros(A * R, dtype=np.int64)
    cols_per_angle: List[np.ndarray] = []
    vals_per_angle: List[np.ndarray] = []
    for a in range(A):
        phi = a * math.pi / A
        cph, sph = math.cos(phi), math.sin(phi)
        p0x, p0y = sb * cph, sb * sph
        ux, uy = -sph, cph
        lox, hix = _slab(p0x, ux, half)
        loy, hiy = _slab(p0y, uy, half)
        tmin = np.maximum(lox, loy)
        tmax = np.minimum(hix, hiy)
        hit = tmax > tmin
        tmin = np.where(hit, tmin, 0.0)
        tmax = np.where(hit, tmax, 0.0)
        parts = [tmin[:, None]]
        if abs(ux) >= 1e-12:
            parts.append((edges[None, :] - p0x[:, None]) / ux)
        if abs(uy) >= 1e-12:
            parts.append((edges[None, :] - p0y[:, None]) / uy)
        parts.append(tmax[:, None])
        t = np.concatenate(parts, axis=1)
        t = np.clip(t, tmin[:, None], tmax[:, None])
        t.sort(axis=1)
        seg = np.diff(t, axis=1)
        mid = 0.5 * (t[:, 1:] + t[:, :-1])
        mx = p0x[:, None] + mid * ux
        my = p0y[:, None] + mid * uy
        c = np.clip(np.floor(mx + half).astype(np.int64), 0, n - 1)
        r = np.clip(np.floor(my + half).astype(np.int64), 0, n - 1)
        keep = seg > min_seg
        counts[a * R:(a + 1) * R] = keep.sum(axis=1)
        cols_per_angle.append((r * n + c)[keep].astype(np.int32))
        vals_per_angle.append(seg[keep])
    row_ptr = np.zeros(A * R + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate(cols_per_angle)
    val = np.concatenate(vals_per_angle)
    return SparseMatrix(A * R, n * n, row_ptr, col, val)


def chord_length_square(phi: float, s: float, half: float) -> float:
    """Length of the line x cos(phi) + y sin(phi) = s inside [-half, half]^2.

    Computed by intersecting the line with the four edges (independent of the
    slab method used by the matrix builder); used to pin row sums.
    """
    c, sn = math.cos(phi), math.sin(phi)
    pts = []
    for xe in (-half, half):
        if abs(sn) > 1e-15:
            y = (s - xe * c) / sn
            if -half - 1e-12 <= y <= half + 1e-12:
                pts.append((xe, y))
    for ye in (-half, half):
        if abs(c) > 1e-15:
            x = (s - ye * sn) / c
            if -half - 1e-12 <= x <= half + 1e-12:
                pts.append((x, ye))
    if len(pts) < 2:
        return 0.0
    best = 0.0
    for i in range(len(pts)):
        for k in range(i + 1, len(pts)):
            best = max(best, math.hypot(pts[i][0] - pts[k][0], pts[i][1] - pts[k][1]))
    return best


def ellipse_phantom(n: int, rng: np.random.Generator, n_ellipses: int = 6) -> np.ndarray:
    """Additive random ellipses (zero background), membership by pixel centre.

    Centre uniform in the disk of radius 0.6*N/2, semi-axes U[0.05N, 0.2N],
    rotation U[0, pi), intensity U[0.5, 4].  Draws that would reach outside
    the field-of-view disk (radius N/2) are rejected.
    """
    half = n / 2.0
    xs = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    X, Y = np.meshgrid(xs, xs)   # X varies along c, Y along r
    img = np.zeros((n, n), dtype=np.float64)
    placed = 0
    while placed < n_ellipses:
        rad = 0.6 * half * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = rad * math.cos(ang), rad * math.sin(ang)
        ax = rng.uniform(0.05 * n, 0.2 * n)
        ay = rng.uniform(0.05 * n, 0.2 * n)
        rot = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.5, 4.0)
        if math.hypot(cx, cy) + max(ax, ay) > half:
            continue
        cr, sr = math.cos(rot), math.sin(rot)
        xr = (X - cx) * cr + (Y - cy) * sr
        yr = -(X - cx) * sr + (Y - cy) * cr
        img += val * ((xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0)
        placed += 1
    return img.reshape(-1)


def disc_phantom(n: int, rng: np.random.Generator) -> np.ndarray:
    """A uniform disc (activity 1, zero background), membership by pixel centre.

    Radius U[0.3, 0.45] * N and centre offset uniform in the disk of radius
    0.05 * N about the image centre, so the disc stays inside the field of view.
    """
    xs = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    X, Y = np.meshgrid(xs, xs)
    rad = rng.uniform(0.3, 0.45) * n
    off = 0.05 * n * math.sqrt(rng.uniform())
    ang = rng.uniform(0.0, 2.0 * math.pi)
    cx, cy = off * math.cos(ang), off * math.sin(ang)
    return ((X - cx) ** 2 + (Y - cy) ** 2 <= rad * rad).astype(np.float64).reshape(-1)


def _column_sums(A: SparseMatrix) -> np.ndarray:
    s = np.zeros(A.n_cols, dtype=np.float64)
    np.add.at(s, A.col, A.val)
    return s


def make_problem(geom: Geometry, seeds: List[int], tc=1e6, rf=0.1,
                 A: Optional[SparseMatrix] = None, tc_range=None, rf_range=None,
                 phantom: str = "ellipses") -> Problem:
    """Phantoms, scaled expected data and Poisson counts for each seed.

    Per seed: rng = default_rng(seed); if ``tc_range``/``rf_range`` are given
    the total counts are 10**U[log10 lo, log10 hi] and the background fraction
    U[lo, hi] (drawn first, in that order); then the phantom ("ellipses" or
    "disc") is drawn.  f_true
    is scaled so that sum(A f_true) = (1 - rf) * TC and gamma_i = rf * TC / m in
    every bin; g = Poisson(A f_true + gamma) from default_rng(seed + 10**6).
    g and gamma are rounded to float32 once, here, so every consumer sees the
    same values.
    """
    if A is None:
        A = siddon_matrix(geom)
    colsum = _column_sums(A)
    m, d = geom.m, geom.d
    B = len(seeds)
    g = np.zeros((B, m), dtype=np.float32)
    gam = np.zeros((B, m), dtype=np.float32)
    ftrue = np.zeros((B, d), dtype=np.float64)
    tcs = np.zeros(B)
    rfs = np.zeros(B)
    # row-wise projection of the truth (input synthesis, FP64)
    rows = np.repeat(np.arange(m), np.diff(A.row_ptr))
    for k, seed in enumerate(seeds):
        rng = np.random.default_rng(seed)
        tck = tc
        rfk = rf
        if tc_range is not None:
            tck = 10.0 ** rng.uniform(math.log10(tc_range[0]), math.log10(tc_range[1]))
        if rf_range is not None:
            rfk = rng.uniform(rf_range[0], rf_range[1])
        if phantom == "ellipses":
            f0 = ellipse_phantom(geom.n, rng)
        elif phantom == "disc":
            f0 = disc_phantom(geom.n, rng)
        else:
            raise ValueError("unknown phantom %r" % phantom)
        f0 *= (1.0 - rfk) * tck / float(colsum @ f0)
        mean = np.zeros(m, dtype=np.float64)
        np.add.at(mean, rows, A.val * f0[A.col])
        gval = rfk * tck / m
        mean += gval
        noise = np.random.default_rng(seed + 10 ** 6)
        g[k] = noise.poisson(mean).astype(np.float32)
        gam[k] = np.float32(gval)
        ftrue[k] = f0
        tcs[k] = tck
        rfs[k] = rfk
    return Problem(geom, A, g, gam, ftrue, tcs, rfs, list(seeds))


# Workload configurations (sizes, counts, parameters).  lambda1 = lambda2 = lambda.
CONFIGS: Dict[str, dict] = {
    "c1_64": dict(geom=Geometry(64, 96, 90), seeds=[1], tc=1e5, rf=0.1,
                  lam=0.05, eps=1e-3, omegas=[0.5], iters=100),
    "c2_128": dict(geom=Geometry(128, 200, 168), seeds=[2], tc=1e6, rf=0.1,
                   lam=0.02, eps=1e-3, omegas=[0.2, 0.5, 1.0], iters=500),
    "c3_128x64": dict(geom=Geometry(128, 200, 168), seeds=list(range(1000, 1064)),
                      tc_range=(1e5, 1e7), rf_range=(0.05, 0.20),
                      lam=0.02, eps=1e-3, omegas=[0.5], iters=300),
    "c4_256x47": dict(geom=Geometry(256, 256, 252), seeds=list(range(3000, 3047)), tc=1e7, rf=0.1,
                      lam=0.01, eps=1e-3, omegas=[1.0], iters=200),
}

_matrix_cache: Dict[Geometry, SparseMatrix] = {}


def cached_matrix(geom: Geometry) -> SparseMatrix:
    if geom not in _matrix_cache:
        _matrix_cache[geom] = siddon_matrix(geom)
    return _matrix_cache[geom]


def config_problem(name: str, n_slices: Optional[int] = None) -> Problem:
    cfg = CONFIGS[name]
    seeds = cfg["seeds"] if n_slices is None else cfg["seeds"][:n_slices]
    return make_problem(cfg["geom"], seeds, tc=cfg.get("tc", 1e6), rf=cfg.get("rf", 0.1),
                        A=cached_matrix(cfg["geom"]), tc_range=cfg.get("tc_range"),
                        rf_range=cfg.get("rf_range"))


# ------------------------------------------------------- Section 4.1 physics ---

@dataclasses.dataclass
class PhysicsProblem:
    """Data with PSF, attenuation, scatter and randoms.  The reconstruction model
    is A = diag(att) G H with G = the Siddon matrix, H the Gaussian PSF of
    `fwhm_px`, att the per-ray attenuation factors, and gamma = scatter + randoms."""
    geom: Geometry
    G: SparseMatrix
    att: np.ndarray      # (m,) attenuation factors exp(-(G mu)_i), FP64
    mu: np.ndarray       # (d,) attenuation coefficient per pixel (per unit path length)
    fwhm_px: float
    g: np.ndarray        # (B, m) float32 counts
    gamma: np.ndarray    # (B, m) float32 scatter + randoms
    f_true: np.ndarray   # (B, d) unblurred truth
    tc: np.ndarray
    seeds: List[int]


def water_disc_mu(geom: Geometry, mu_per_cm: float = 0.096, fov_mm: float = 300.0) -> np.ndarray:
    """Uniform water (0.096 / cm, Section 4.1) on the field-of-view disk of radius N/2, in
    units of the geometry's pixel side (a pixel is fov_mm / N wide)."""
    n = geom.n
    c = np.arange(n) - (n - 1) / 2.0
    y, x = np.meshgrid(c, c, indexing="ij")
    inside = (x * x + y * y) <= (n / 2.0) ** 2
    return np.where(inside, mu_per_cm * (fov_mm / n) / 10.0, 0.0).ravel()


def make_physics_problem(geom: Geometry, seeds: List[int], tc=1e6, sf=0.25, rf=0.25,
                         fwhm_mm=6.59, fov_mm=300.0, scatter_fwhm_px=None,
                         G: Optional[SparseMatrix] = None, phantom: str = "ellipses") -> PhysicsProblem:
    """Counts after Section 4.1's simulation recipe, per seed:

    * the truth (random ellipses) blurred by the Gaussian PSF (FWHM fwhm_mm, pixel
      fov_mm / N; scipy.ndimage.gaussian_filter, zero outside the image, truncated at 3
      sigma) and forward projected through G, then attenuated: Tc = att * G (PSF f);
    * scatter: the projection of a heavily smoothed truth (FWHM N/4 pixels), scaled so
      that SF = Sc / (Tc + Sc);
    * randoms: uniform, scaled so that RF = Rc / (Tc + Sc + Rc);
    * everything scaled so that TC = Tc + Sc + Rc; g = Poisson(Tc + Sc + Rc).
    The attenuation map is a water disc over the field of view, the same for every seed
    (so a batch shares one system matrix).
    """
    from scipy.ndimage import gaussian_filter
    if G is None:
        G = siddon_matrix(geom)
    m, d, n = geom.m, geom.d, geom.n
    rows = np.repeat(np.arange(m), np.diff(G.row_ptr))

    def project(x):
        out = np.zeros(m)
        np.add.at(out, rows, G.val * x[G.col])
        return out

    mu = water_disc_mu(geom, fov_mm=fov_mm)
    att = np.exp(-project(mu))
    fwhm_px = fwhm_mm / (fov_mm / n)
    to_sigma = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    s_fwhm = n / 4.0 if scatter_fwhm_px is None else scatter_fwhm_px
    B = len(seeds)
    g = np.zeros((B, m), dtype=np.float32)
    gam = np.zeros((B, m), dtype=np.float32)
    ftrue = np.zeros((B, d))
    for k, seed in enumerate(seeds):
        rng = np.random.default_rng(seed)
        f0 = ellipse_phantom(n, rng) if phantom == "ellipses" else disc_phantom(n, rng)
        img = f0.reshape(n, n)
        blurred = gaussian_filter(img, fwhm_px * to_sigma, mode="constant", truncate=3.0).ravel()
        smooth = gaussian_filter(img, s_fwhm * to_sigma, mode="constant", truncate=3.0).ravel()
        T = att * project(blurred)
        S = project(smooth)
        S *= (sf / (1.0 - sf)) * T.sum() / S.sum()
        Rc = (rf / (1.0 - rf)) * (T.sum() + S.sum())
        R = np.full(m, Rc / m)
        scale = tc / (T.sum() + S.sum() + R.sum())
        f0 = f0 * scale
        T, S, R = T * scale, S * scale, R * scale
        noise = np.random.default_rng(seed + 10 ** 6)
        g[k] = noise.poisson(T + S + R).astype(np.float32)
        gam[k] = (S + R).astype(np.float32)
        ftrue[k] = f0
    return PhysicsProblem(geom, G, att, mu, fwhm_px, g, gam, ftrue, np.full(B, float(tc)), list(seeds))
