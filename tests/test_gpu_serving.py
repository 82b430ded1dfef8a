"""Continuous-batching server: results alone vs in a mix of sizes, parameters and
budgets arriving while others run; admission under an HBM budget; error paths."""
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2409_13344_amd import appga as ap  # noqa: E402
from paper_2409_13344_amd import synth  # noqa: E402


def say(msg):
    print("[gpu-serving] " + msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    ctx = ap.appga_create(0)
    small = synth.Geometry(64, 96, 90)
    mid = synth.Geometry(128, 200, 168)
    mats = {}
    probs = {}
    for name, geom, seeds in (("small", small, [11, 12, 13, 14, 15]),
                              ("mid", mid, [21, 22, 23, 24, 25])):
        pr = synth.make_problem(geom, seeds, tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
        probs[name] = pr
        mats[name] = ap.load_matrix(ctx, pr.A, geom, "f32")
    yield ctx, mats, probs
    for m in mats.values():
        ap.appga_free_system_matrix(ctx, m)
    ap.appga_destroy(ctx)


def _requests(probs):
    rng = np.random.default_rng(77)
    reqs = []
    for i in range(10):
        name = "small" if i % 2 == 0 else "mid"
        pr = probs[name]
        b = i // 2
        p = ap.make_params(lam=float(rng.uniform(0.005, 0.1)), eps=1e-3,
                           omega=float(rng.choice([0.3, 0.6, 1.0])),
                           iterations=int(rng.integers(20, 90)))
        reqs.append((name, b, p))
    return reqs


def test_served_results_match_solo_and_mix(setup):
    ctx, mats, probs = setup
    reqs = _requests(probs)
    srv = ap.appga_server_start(ctx, 1 << 34, 64)
    try:
        # each request alone in the server
        alone = []
        for name, b, p in reqs[:4]:
            pr = probs[name]
            t = ap.appga_submit(srv, mats[name], pr.g[b], pr.gamma[b], p)
            f, st = ap.appga_wait(srv, t, pr.geom.d, 60000)
            alone.append(f)
            assert st["iterations_done"] == p.iterations
        # the same and more requests, arriving while others run
        tickets = [None] * len(reqs)

        def submitter():
            for i, (name, b, p) in enumerate(reqs):
                pr = probs[name]
                tickets[i] = ap.appga_submit(srv, mats[name], pr.g[b], pr.gamma[b], p)
                time.sleep(0.002)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        mixed = []
        for i, (name, b, p) in enumerate(reqs):
            f, st = ap.appga_wait(srv, tickets[i], probs[name].geom.d, 60000)
            assert st["iterations_done"] == p.iterations
            assert st["seconds"] > 0
            assert st["guard_clamps"] == 0
            mixed.append(f)
    finally:
        ap.appga_server_stop(srv)
    for i in range(4):
        # lanes are independent: alone and in the mix are the same computation
        np.testing.assert_array_equal(mixed[i], alone[i])
    # FP64 oracle: 1e-5, or the problem's own floor where it amplifies an
    # FP32-size perturbation of the data (1e-7 relative) beyond that
    def oracle_pair(i):
        name, b, p = reqs[i]
        pr = probs[name]
        run = lambda g: oracle.appga(pr.A, pr.geom.n, pr.geom.n_angles, g, pr.gamma[b], p.lambda1,
                                     p.lambda2, p.eps, p.omega, p.iterations)["f"]
        g = pr.g[b].astype(np.float64)
        pert = g * (1.0 + 1e-7 * np.random.default_rng(1000 + i).standard_normal(g.shape))
        f0 = run(g)
        return f0, rel_l2(run(pert), f0)

    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(oracle_pair, range(len(reqs))))
    # the batched session path runs the same kernels on the same lane layout
    # (a batch of two copies, so that it takes the lane path rather than B = 1)
    for i, (name, b, p) in enumerate(reqs):
        pr = probs[name]
        fb, _ = ap.appga_reconstruct_batch(ctx, mats[name], pr.geom.d, pr.g[[b, b]],
                                           pr.gamma[[b, b]], [p, p])
        err = rel_l2(mixed[i], fb[0])
        say("request %d (%s): served vs batched session %.2e" % (i, name, err))
        # the server sums ACTc on the host, the session on the device: a last-bit
        # difference of the initial image, amplified by the problem's floor
        assert err <= max(1e-6, 4.0 * refs[i][1])
    for i, (name, b, p) in enumerate(reqs):
        ref, floor = refs[i]
        err = rel_l2(mixed[i], ref)
        tol = max(1e-5, 4.0 * floor)
        say("request %d (%s, omega %.1f, K %d): vs FP64 oracle %.2e (floor %.2e, tol %.2e)"
            % (i, name, p.omega, p.iterations, err, floor, tol))
        assert err <= tol


def test_budget_admits_one_pool_at_a_time(setup):
    ctx, mats, probs = setup
    # a budget that holds either pool but not both: the second geometry waits
    # until the first pool drains and is freed
    big = ap.appga_server_footprint(mats["mid"])
    small = ap.appga_server_footprint(mats["small"])
    assert big > small > 0
    srv = ap.appga_server_start(ctx, big + small // 2, 8)
    try:
        ts = []
        for i in range(6):
            name = "mid" if i < 3 else "small"
            pr = probs[name]
            p = ap.make_params(lam=0.02, omega=0.5, iterations=15)
            ts.append((name, ap.appga_submit(srv, mats[name], pr.g[i % 5], pr.gamma[i % 5], p)))
        for name, t in ts:
            f, st = ap.appga_wait(srv, t, probs[name].geom.d, 60000)
            assert st["iterations_done"] == 15
            assert np.isfinite(f).all()
    finally:
        ap.appga_server_stop(srv)


def test_server_errors(setup):
    ctx, mats, probs = setup
    srv = ap.appga_server_start(ctx, 1 << 32, 4)
    tiny = ap.appga_server_start(ctx, 1 << 20, 4)
    try:
        pr = probs["small"]
        with pytest.raises(ap.AppgaError) as ei:    # the pool can never fit the budget
            ap.appga_submit(tiny, mats["small"], pr.g[0], pr.gamma[0], ap.make_params(iterations=5))
        assert ei.value.status == -4
        with pytest.raises(ap.AppgaError) as ei:
            ap.appga_wait(srv, 12345, pr.geom.d, 10)
        assert ei.value.status == -8
        with pytest.raises(ap.AppgaError) as ei:
            ap.appga_submit(srv, mats["small"], pr.g[0], pr.gamma[0],
                            ap.make_params(eps=-1.0, iterations=5))
        assert ei.value.status == -3
        with pytest.raises(ap.AppgaError) as ei:
            ap.appga_submit(srv, mats["small"], pr.g[0], pr.gamma[0],
                            ap.make_params(precond=ap.APPGA_PRECOND_FIXED, fixed_p=1e-3,
                                           iterations=5))
        assert ei.value.status == -1
        t = ap.appga_submit(srv, mats["small"], pr.g[0], pr.gamma[0],
                            ap.make_params(lam=0.02, iterations=400))
        with pytest.raises(ap.AppgaError) as ei:
            ap.appga_free_system_matrix(ctx, mats["small"])       # in use
        assert ei.value.status == -7
        f, st = ap.appga_wait(srv, t, pr.geom.d, 60000)
        assert st["iterations_done"] == 400
    finally:
        ap.appga_server_stop(srv)
        ap.appga_server_stop(tiny)
