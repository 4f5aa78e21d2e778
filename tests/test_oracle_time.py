"""Pins of the oracle's time stepping (paper Eq. 2 and Algorithm 1; source
injection of Section IV-D; ghost layer of Section IV-B).

The pins are properties the discrete method must have, derived by hand:
the one-step impulse response, the discrete plane-wave dispersion relation
on a periodic grid, conservation of the discrete energy, source-receiver
reciprocity, and a brute-force run with an independently built operator."""
import math

import numpy as np
import pytest

from _pins import golden_coefficients, kron_laplacian, rel_l2


def _symbol(kh, c):
    """c0 + 2 sum_m c_m cos(m kh) for the published weights."""
    return float(c[0]) + 2.0 * sum(float(c[m]) * math.cos(m * kh) for m in range(1, 5))


def test_impulse_response_one_step(oracle_lib):
    # u^0 = delta at P, u^{-1} = 0: one step gives exactly 25 non-zeros:
    # 2 + k_P c0 sum_a 1/h_a^2 at P and k_Q c_m / h_a^2 at Q = P +- m e_a.
    c = golden_coefficients()
    nz, ny, nx = 11, 12, 13
    h = (1.5, 2.5, 3.5)  # dx, dy, dz
    rng = np.random.default_rng(3)
    k = rng.uniform(0.1, 0.3, size=(nz, ny, nx))
    P = (5, 6, 7)
    a0 = np.zeros((nz, ny, nx))
    a0[P] = 1.0
    cur, prev, _ = oracle_lib.run(k, h, 1, a_cur=a0)
    assert np.array_equal(prev, a0)
    expect = np.zeros_like(a0)
    inv = {0: 1 / h[2] ** 2, 1: 1 / h[1] ** 2, 2: 1 / h[0] ** 2}  # by array axis z, y, x
    expect[P] = 2.0 + k[P] * float(c[0]) * sum(inv.values())
    for ax in range(3):
        for m in range(1, 5):
            for sgn in (-1, 1):
                Q = list(P)
                Q[ax] += sgn * m
                Q = tuple(Q)
                expect[Q] = k[Q] * float(c[m]) * inv[ax]
    assert np.count_nonzero(cur) == 25
    assert np.allclose(cur, expect, rtol=1e-14, atol=0)


def test_plane_wave_dispersion_periodic(oracle_lib):
    # u^n = cos(kappa . x - omega n dt) solves the scheme exactly on a torus
    # when 4 sin^2(omega dt / 2) = K sum_a (-1/h_a^2)(c0 + 2 sum c_m cos(m kappa_a h_a)).
    c = golden_coefficients()
    nz, ny, nx = 10, 12, 16
    h = (7.0, 9.0, 11.0)  # dx, dy, dz
    j = (3, 2, 1)  # wave numbers along x, y, z
    kap = [2 * math.pi * j[0] / (nx * h[0]), 2 * math.pi * j[1] / (ny * h[1]),
           2 * math.pi * j[2] / (nz * h[2])]
    K = 0.9 * 4.0 / (2048 / 315 * sum(1 / hh ** 2 for hh in h))  # stable, 0.9 of the limit
    lam = -sum(_symbol(kap[a] * h[a], c) / h[a] ** 2 for a in range(3))
    wdt = 2.0 * math.asin(math.sqrt(K * lam) / 2.0)
    z = np.arange(nz)[:, None, None] * h[2]
    y = np.arange(ny)[None, :, None] * h[1]
    x = np.arange(nx)[None, None, :] * h[0]
    phase = kap[0] * x + kap[1] * y + kap[2] * z
    u0 = np.cos(phase) * np.ones((nz, ny, nx))
    um1 = np.cos(phase + wdt) * np.ones((nz, ny, nx))
    k = np.full((nz, ny, nx), K)
    nsteps = 300
    cur, prev, _ = oracle_lib.run(k, h, nsteps, a_cur=u0, a_prev=um1, bc=oracle_lib.BC_PERIODIC)
    ref = np.cos(phase - wdt * nsteps)
    assert np.abs(cur - ref).max() < 1e-11
    # a 1e-6 relative error in any weight would move the phase measurably
    lam_bad = lam * (1 + 1e-6)
    wdt_bad = 2.0 * math.asin(math.sqrt(K * lam_bad) / 2.0)
    assert np.abs(np.cos(phase - wdt_bad * nsteps) - ref).max() > 1e-8


def _energy(oracle_lib, k, h, a_new, a_old):
    pad = np.zeros(tuple(s + 8 for s in a_old.shape))
    pad[4:-4, 4:-4, 4:-4] = a_old
    L = oracle_lib.laplacian(pad, h)
    return float(np.sum((a_new - a_old) ** 2 / k) - np.sum(a_new * L))


def test_discrete_energy_conserved(oracle_lib):
    # With a symmetric L (zero ghost layer), heterogeneous k and no sponge or
    # source, E = sum (u^{n+1}-u^n)^2 / k - sum u^{n+1} L u^n is invariant.
    rng = np.random.default_rng(11)
    nz, ny, nx = 14, 15, 16
    h = (10.0, 12.0, 9.0)
    lim = 4.0 / (2048 / 315 * sum(1 / hh ** 2 for hh in h))
    k = rng.uniform(0.2, 0.85, size=(nz, ny, nx)) * lim
    a_prev = rng.standard_normal((nz, ny, nx))
    a_cur = a_prev + 0.1 * rng.standard_normal((nz, ny, nx))
    e = []
    for _ in range(40):
        new, old, _ = oracle_lib.run(k, h, 1, a_cur=a_cur, a_prev=a_prev)
        e.append(_energy(oracle_lib, k, h, new, old))
        a_cur, a_prev = new, old
    e = np.array(e)
    assert e[0] > 0
    assert np.abs(e / e[0] - 1).max() < 1e-12


def _reciprocity_pair(oracle_lib, W):
    rng = np.random.default_rng(5 + W)
    nz, ny, nx = 22, 20, 18
    h = (10.0, 10.0, 10.0)
    dt = 1.2e-3
    v = rng.uniform(1500.0, 3000.0, size=(nz, ny, nx))
    k = (v * dt) ** 2
    A, B = (8, 9, 7), (13, 11, 10)
    nt = 160
    w = np.sin(np.arange(nt) * 0.37) * np.exp(-((np.arange(nt) - 20) / 8.0) ** 2)
    _, _, tAB = oracle_lib.run(k, h, nt, s=k[A] * w, src=A, rec=[B], sponge_width=W,
                               sponge_alpha=0.05)
    _, _, tBA = oracle_lib.run(k, h, nt, s=k[B] * w, src=B, rec=[A], sponge_width=W,
                               sponge_alpha=0.05)
    return tAB[:, 0], tBA[:, 0]


@pytest.mark.parametrize("W", [0, 4])
def test_source_receiver_reciprocity(oracle_lib, W):
    # With Eq. 2 scaling (injected value k_src * w) the response is
    # symmetric in source and receiver; with the sponge this holds for
    # points outside the damping strip (G = 1 there).
    tab, tba = _reciprocity_pair(oracle_lib, W)
    assert np.abs(tab).max() > 0
    assert np.abs(tab - tba).max() <= 1e-12 * np.abs(tab).max()


def test_brute_force_kronecker_recurrence(oracle_lib):
    # Tiny heterogeneous problem with sponge, source and receivers against a
    # recurrence on an explicitly assembled sparse operator.
    c = golden_coefficients()
    rng = np.random.default_rng(23)
    nz, ny, nx = 9, 7, 11
    h = (9.0, 11.0, 7.0)
    lim = 4.0 / (2048 / 315 * sum(1 / hh ** 2 for hh in h))
    k = rng.uniform(0.3, 0.8, size=(nz, ny, nx)) * lim
    W, alpha = 3, 0.2
    nt = 37
    s = rng.standard_normal(nt)
    src = (4, 3, 5)
    rec = np.array([[0, 0, 0], [4, 3, 5], [8, 6, 10], [2, 5, 1]], dtype=np.int32)
    cur, prev, tr = oracle_lib.run(k, h, nt, s=s, src=src, rec=rec, sponge_width=W,
                                   sponge_alpha=alpha)
    L = kron_laplacian(nz, ny, nx, h, c)

    def prof(n):
        d = np.minimum(np.arange(n), n - 1 - np.arange(n))
        return np.where(d < W, np.exp(-(alpha * (W - d)) ** 2), 1.0)

    G = (prof(nz)[:, None, None] * prof(ny)[None, :, None] * prof(nx)[None, None, :]).ravel()
    kk = k.ravel()
    u, up = np.zeros(kk.size), np.zeros(kk.size)
    si = np.ravel_multi_index(src, (nz, ny, nx))
    ri = np.ravel_multi_index(rec.T, (nz, ny, nx))
    trb = np.zeros((nt, len(rec)))
    for n in range(nt):
        un = G * (2 * u - G * up + kk * (L @ u))
        un[si] += s[n]
        trb[n] = un[ri]
        up, u = u, un
    assert rel_l2(cur.ravel(), u) < 1e-13
    assert rel_l2(prev.ravel(), up) < 1e-13
    assert rel_l2(tr, trb) < 1e-13


def test_restart_is_bitwise(oracle_lib):
    rng = np.random.default_rng(31)
    nz, ny, nx = 12, 13, 14
    h = (10.0, 10.0, 10.0)
    k = rng.uniform(0.01, 0.05, size=(nz, ny, nx)) * 100
    s = rng.standard_normal(60)
    rec = [[1, 2, 3], [6, 6, 6]]
    a1, p1, t1 = oracle_lib.run(k, h, 60, s=s, src=(6, 6, 7), rec=rec, sponge_width=3,
                                sponge_alpha=0.1)
    a2, p2, t2 = oracle_lib.run(k, h, 25, s=s, src=(6, 6, 7), rec=rec, sponge_width=3,
                                sponge_alpha=0.1)
    a3, p3, t3 = oracle_lib.run(k, h, 35, s=s[25:], src=(6, 6, 7), rec=rec, a_cur=a2,
                                a_prev=p2, sponge_width=3, sponge_alpha=0.1)
    assert np.array_equal(a1, a3) and np.array_equal(p1, p3)
    assert np.array_equal(t1, np.concatenate([t2, t3]))


def test_segmented_run_is_bitwise(oracle_lib):
    # the segmented form used for long runs (progress between segments)
    # returns exactly what one call returns, including a ragged last segment
    rng = np.random.default_rng(32)
    k = rng.uniform(0.5, 2.0, size=(10, 11, 12))
    s = rng.standard_normal(47)
    kw = dict(src=(5, 5, 6), rec=[[1, 2, 3], [8, 9, 10]], sponge_width=3, sponge_alpha=0.1)
    a1, p1, t1 = oracle_lib.run(k, (10.0, 10.0, 10.0), 47, s=s, **kw)
    seen = []
    a2, p2, t2, sec = oracle_lib.run_segments(k, (10.0, 10.0, 10.0), 47, 10, s=s,
                                              progress=lambda d, n, t: seen.append(d), **kw)
    assert seen == [10, 20, 30, 40, 47] and sec > 0
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2) and np.array_equal(t1, t2)


def test_thread_count_invariance(oracle_lib):
    rng = np.random.default_rng(41)
    k = rng.uniform(0.5, 1.0, size=(16, 9, 10)) * 10
    s = rng.standard_normal(20)
    r1 = oracle_lib.run(k, (10.0, 10.0, 10.0), 20, s=s, src=(3, 4, 5), nthreads=1)
    r4 = oracle_lib.run(k, (10.0, 10.0, 10.0), 20, s=s, src=(3, 4, 5), nthreads=4)
    assert np.array_equal(r1[0], r4[0]) and np.array_equal(r1[1], r4[1])


def test_sponge_profile_definition(oracle_lib):
    g = oracle_lib.sponge_profile(60, 20, 0.015)
    assert g[0] == pytest.approx(math.exp(-0.09), rel=1e-15)
    assert g[-1] == g[0]
    assert np.all(g[20:40] == 1.0)
    assert np.all(np.diff(g[:21]) > 0)
    assert np.array_equal(g, g[::-1])
    assert np.all(oracle_lib.sponge_profile(17, 0, 0.3) == 1.0)


def test_sponge_damps_both_time_levels(oracle_lib):
    # On a one-cell grid (zero ghosts all round) the Laplacian is its centre
    # term alone, so the scheme is the scalar recurrence
    #     u^{n+1} = G ((2 + K lam) u^n - G u^{n-1}) + s_n,
    # G the product of the three axis factors.  With one source value at
    # step 0, damping both time levels by G gives u^{n+1} = G^n w^{n+1}, w
    # the undamped solution: trace row n of the sponge run is G^n times that
    # of the plain run.  Damping only the new level, or only the old one,
    # breaks this identity.
    h = (10.0, 12.0, 9.0)
    k = np.full((1, 1, 1), 7.0)
    s = np.zeros(40)
    s[0] = 1.0
    alpha, width = 0.37, 1
    plain = oracle_lib.run(k, h, 40, s=s, src=(0, 0, 0), rec=[(0, 0, 0)])[2][:, 0]
    damped = oracle_lib.run(k, h, 40, s=s, src=(0, 0, 0), rec=[(0, 0, 0)], sponge_width=width,
                            sponge_alpha=alpha)[2][:, 0]
    g = oracle_lib.sponge_profile(1, width, alpha)[0] ** 3
    n = np.arange(40)
    assert np.abs(plain).max() > 0.5  # an oscillation, not a decay to zero
    np.testing.assert_allclose(damped, g ** n * plain, rtol=1e-12, atol=1e-14)
    # the profile's value there: the face cell of a one-cell strip
    assert g == pytest.approx(math.exp(-3 * (alpha * width) ** 2), rel=1e-14)


def test_sponge_width_zero_is_plain_scheme(oracle_lib):
    rng = np.random.default_rng(2)
    k = rng.uniform(1.0, 3.0, size=(10, 11, 12))
    s = rng.standard_normal(15)
    a = oracle_lib.run(k, (10.0, 10.0, 10.0), 15, s=s, src=(5, 5, 5))
    b = oracle_lib.run(k, (10.0, 10.0, 10.0), 15, s=s, src=(5, 5, 5), sponge_width=0,
                       sponge_alpha=0.7)
    assert np.array_equal(a[0], b[0])


def test_sponge_removes_energy(oracle_lib):
    # A pulse in the middle radiates into the strip and is damped there.
    nz = ny = nx = 30
    h = (10.0, 10.0, 10.0)
    lim = 4.0 / (2048 / 315 * 3 / 100.0)
    k = np.full((nz, ny, nx), 0.5 * lim)
    z, y, x = np.meshgrid(*(np.arange(n) - 14.5 for n in (nz, ny, nx)), indexing="ij")
    a0 = np.exp(-(x * x + y * y + z * z) / 8.0)
    e0 = _energy(oracle_lib, k, h, *oracle_lib.run(k, h, 1, a_cur=a0, a_prev=a0)[:2])
    cur, prev, _ = oracle_lib.run(k, h, 200, a_cur=a0, a_prev=a0, sponge_width=8,
                                  sponge_alpha=0.08)
    e1 = _energy(oracle_lib, k, h, cur, prev)
    assert 0 < e1 < 0.2 * e0


def test_step_points_matches_run(oracle_lib):
    from paper_2204_03775_amd.inputs import random_problem

    p = random_problem(13, 11, 9, 12, seed=8, sponge_width=3)
    k = p.k64()
    cur, prev, _ = oracle_lib.run(k, p.h, 11, s=p.s, src=p.src, sponge_width=3,
                                  sponge_alpha=p.sponge_alpha)
    c32, p32, k32 = cur.astype(np.float32), prev.astype(np.float32), k.astype(np.float32)
    nxt, _, _ = oracle_lib.run(k32.astype(np.float64), p.h, 1, s=p.s[11:], src=p.src,
                               a_cur=c32.astype(np.float64), a_prev=p32.astype(np.float64),
                               sponge_width=3, sponge_alpha=p.sponge_alpha)
    pts = np.argwhere(np.ones(p.shape, dtype=bool)).astype(np.int32)
    got = oracle_lib.step_points(k32, c32, p32, p.h, pts, sponge_width=3,
                                 sponge_alpha=p.sponge_alpha, src=p.src, src_value=p.s[11])
    assert np.abs(got - nxt.ravel()).max() <= 1e-13 * np.abs(nxt).max()


def test_stability_limit(oracle_lib):
    # Leapfrog with a symmetric operator is stable iff K * lambda_max <= 4,
    # lambda_max = (2048/315) sum_a 1/h_a^2 the largest eigenvalue of -lap
    # (the Nyquist mode, present on an even periodic grid).  Just below the
    # limit random data stay bounded; just above, the Nyquist mode grows
    # like (1 + 2 sqrt(delta))^n.  This pins the limit the library checks
    # at init and the workloads' dt rule.
    from paper_2204_03775_amd.inputs import SYMBOL_MAX, stable_courant_limit

    h = (9.0, 11.0, 7.0)
    lam_max = SYMBOL_MAX * sum(1.0 / hh ** 2 for hh in h)
    k_lim = 4.0 / lam_max
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((12, 14, 16))
    peaks = {}
    for f in (0.98, 1.01):
        k = np.full(u0.shape, f * k_lim)
        cur, _, _ = oracle_lib.run(k, h, 250, a_cur=u0, a_prev=u0, bc=oracle_lib.BC_PERIODIC)
        peaks[f] = np.abs(cur).max() / np.abs(u0).max()
    assert peaks[0.98] < 50.0, peaks
    assert peaks[1.01] > 1e6, peaks
    # the cubic-grid Courant limit used for dt: v dt / h <= 2 / sqrt(3 * 2048/315)
    assert stable_courant_limit(3) == pytest.approx(2.0 / math.sqrt(3 * 2048 / 315), rel=1e-15)
    assert stable_courant_limit(3) ** 2 * 3 * SYMBOL_MAX == pytest.approx(4.0, rel=1e-14)
