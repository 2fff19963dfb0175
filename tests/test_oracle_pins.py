"""Pins of the FP64 oracle against mathematics that does not come from the oracle.

The paper prints no numbers for its acoustic isotropic kernel (Sec. 4.5, Fig. 8 holds
only speedups), so every pin here is a closed form, an exact invariant, a textbook
special case or brute force on a tiny grid:

* the 9-point weights are re-derived here from moment conditions, not read from the
  oracle, and the oracle's operator must be exact on polynomials of degree <= 9 and
  fail at degree 10;
* on a periodic grid the operator must equal its Fourier symbol applied by numpy's FFT;
* brute-force matrices of the operator must be symmetric, translation invariant
  (periodic) and have the 25-point star support;
* a discrete plane wave with the closed-form numerical dispersion relation must
  propagate exactly, and the leapfrog stability limit must sit where theory puts it;
* the discrete energy is conserved without damping and dissipates by the exact
  identity with the sponge; source-receiver reciprocity holds; mirror symmetry is
  bitwise; pausing and resuming is bitwise;
* the Ricker wavelet and the sponge profile meet their closed-form properties.
"""
from fractions import Fraction

import numpy as np
import pytest

from workloads import layered_velocity, smooth_velocity, random_field
from bitwise import same_bits

H = 4


# ----------------------------------------------------------------- helpers

def derived_weights():
    """Symmetric 9-point second-derivative weights from the moment conditions
    sum_m c_m m^p = 2*delta_{p,2} (p = 0,2,4,6,8), solved exactly in rationals."""
    # unknowns c0..c4; rows p = 0,2,4,6,8
    A = [[Fraction(1 if p == 0 else 0)] + [Fraction(2 * m ** p) for m in range(1, 5)]
         for p in (0, 2, 4, 6, 8)]
    b = [Fraction(2 if p == 2 else 0) for p in (0, 2, 4, 6, 8)]
    n = 5
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def symbol(theta, c):
    """-(Fourier symbol) of the 1-D operator on unit spacing: s(theta) >= 0."""
    return -float(c[0]) - 2.0 * sum(float(c[m]) * np.cos(m * theta) for m in range(1, 5))


def box_from(fun, nx, ny, nz, d, origin):
    """Evaluate fun(x,y,z) on every point of the padded box, halo included."""
    k, j, i = np.meshgrid(np.arange(-H, nz + H), np.arange(-H, ny + H),
                          np.arange(-H, nx + H), indexing="ij")
    x = origin[0] + i * d[0]
    y = origin[1] + j * d[1]
    z = origin[2] + k * d[2]
    return fun(x, y, z), (x, y, z)


def energy(ora, up, u, un, q, d, periodic):
    """I^n = sum (u^{n+1}-u^n)^2/q - sum u^{n+1} L u^n."""
    b = ora.to_box(u)
    if periodic:
        ora.fill_halo_periodic(b)
    Lu = ora.laplacian(b, d)
    return np.sum((un - u) ** 2 / q) - np.sum(un * Lu)


# ----------------------------------------------------------------- weights

def test_derived_weights_are_the_textbook_8th_order_set():
    c = derived_weights()
    assert c == [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315),
                 Fraction(-1, 560)]


@pytest.mark.parametrize("deg", range(0, 10))
def test_laplacian_exact_on_polynomials(ora, deg):
    """Each 1-D 9-point operator is exact on polynomials of degree <= 9, so L is exact
    on x^a y^b z^c with a, b, c <= 9 (exercises each axis and its spacing)."""
    nx, ny, nz = 7, 6, 5
    d = (0.11, 0.09, 0.13)
    rng = np.random.default_rng(deg)
    coef = rng.uniform(-1, 1, size=3)
    p = [deg, max(deg - 1, 0), max(deg - 2, 0)]

    def f(x, y, z):
        return coef[0] * x ** p[0] + coef[1] * y ** p[1] + coef[2] * (x * 0 + 1) * z ** p[2] \
            + 0.3 * x ** min(deg, 3) * y ** min(deg, 2)

    def lap(x, y, z):
        def d2(t, n):
            return n * (n - 1) * t ** (n - 2) if n >= 2 else 0 * t
        out = coef[0] * d2(x, p[0]) + coef[1] * d2(y, p[1]) + coef[2] * d2(z, p[2])
        a, bb = min(deg, 3), min(deg, 2)
        out = out + 0.3 * (d2(x, a) * y ** bb + x ** a * d2(y, bb))
        return out

    u, (x, y, z) = box_from(f, nx, ny, nz, d, origin=(-0.3, -0.25, -0.35))
    got = ora.laplacian(u, d)
    want = lap(x, y, z)[H:-H, H:-H, H:-H]
    scale = max(1.0, np.abs(want).max(), np.abs(u).max() / min(d) ** 2 * 1e-3)
    assert np.abs(got - want).max() <= 1e-9 * scale


def test_laplacian_not_exact_at_degree_10(ora):
    nx = ny = nz = 5
    d = (0.1, 0.1, 0.1)
    u, (x, y, z) = box_from(lambda x, y, z: x ** 10, nx, ny, nz, d, origin=(0.1, 0, 0))
    got = ora.laplacian(u, d)
    want = (90 * x ** 8)[H:-H, H:-H, H:-H]
    # truncation error of the 8th-order operator on x^10 is c*h^8*10!/... : far above rounding
    err = np.abs(got - want).max()
    assert err > 1e-6 * np.abs(want).max()
    # and it is the h^8 term: 10!/8! * (-1/630) * ... check sign and order of magnitude only
    assert err < 1e-1 * np.abs(want).max()


# ----------------------------------------------------------------- spectral / brute force

@pytest.mark.parametrize("shape,d", [((8, 9, 12), (10.0, 7.0, 13.0)),
                                     ((5, 6, 4), (1.0, 2.0, 0.5))])
def test_periodic_laplacian_matches_fft_symbol(ora, shape, d):
    """On a periodic grid L is diagonal in Fourier space with eigenvalue
    -sum_a s(2 pi k_a/n_a)/d_a^2 (short periods alias the far weights, which the
    symbol accounts for automatically)."""
    nx, ny, nz = shape
    c = derived_weights()
    u = random_field((nz, ny, nx), seed=11).astype(np.float64)
    b = ora.fill_halo_periodic(ora.to_box(u))
    got = ora.laplacian(b, d)
    tz = 2 * np.pi * np.fft.fftfreq(nz)
    ty = 2 * np.pi * np.fft.fftfreq(ny)
    tx = 2 * np.pi * np.fft.fftfreq(nx)
    K = (symbol(tz, c)[:, None, None] / d[2] ** 2 + symbol(ty, c)[None, :, None] / d[1] ** 2
         + symbol(tx, c)[None, None, :] / d[0] ** 2)
    want = np.real(np.fft.ifftn(-K * np.fft.fftn(u)))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def _operator_matrix(ora, shape, d, periodic):
    nx, ny, nz = shape
    n = nx * ny * nz
    M = np.zeros((n, n))
    for p in range(n):
        e = np.zeros(n)
        e[p] = 1.0
        b = ora.to_box(e.reshape(nz, ny, nx))
        if periodic:
            ora.fill_halo_periodic(b)
        M[:, p] = ora.laplacian(b, d).ravel()
    return M


def test_operator_matrix_symmetric_and_translation_invariant(ora):
    shape, d = (6, 5, 7), (1.0, 1.3, 0.8)
    nx, ny, nz = shape
    for periodic in (False, True):
        M = _operator_matrix(ora, shape, d, periodic)
        assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
        if periodic:
            assert np.abs(M.sum(axis=1)).max() <= 1e-12 * np.abs(M).max()
            # commutes with the cyclic shift along each axis
            idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
            for ax in range(3):
                P = np.zeros_like(M)
                P[np.roll(idx, 1, axis=ax).ravel(), idx.ravel()] = 1.0
                assert np.abs(P @ M - M @ P).max() <= 1e-12 * np.abs(M).max()


def test_operator_has_25_point_star_support(ora):
    shape, d = (9, 9, 9), (1.0, 1.0, 1.0)
    M = _operator_matrix(ora, shape, d, periodic=False)
    centre = (4 * 9 + 4) * 9 + 4
    row = M[centre].reshape(9, 9, 9)
    nz_idx = set(zip(*np.nonzero(row)))
    star = {(4, 4, 4)}
    for m in range(1, 5):
        for s in (-m, m):
            star |= {(4 + s, 4, 4), (4, 4 + s, 4), (4, 4, 4 + s)}
    assert nz_idx == star and len(star) == 25


# ----------------------------------------------------------------- time stepping

def test_plane_wave_propagates_with_discrete_dispersion(ora):
    """cos(k.x - w t) with sin(w dt/2) = (v dt/2) sqrt(K(k)) solves the leapfrog
    scheme exactly on a periodic grid."""
    nx, ny, nz = 16, 12, 10
    d = (10.0, 12.0, 8.0)
    v0 = 1800.0
    v = np.full((nz, ny, nx), v0, dtype=np.float32)
    dt = ora.cfl_dt(v, min(d))
    c = derived_weights()
    kv = (2 * np.pi * 2 / (nx * d[0]), 2 * np.pi * 1 / (ny * d[1]), 2 * np.pi * 3 / (nz * d[2]))
    K = sum(symbol(kv[a] * d[a], c) / d[a] ** 2 for a in range(3))
    omega = 2.0 / dt * np.arcsin(0.5 * v0 * dt * np.sqrt(K))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = kv[0] * i * d[0] + kv[1] * j * d[1] + kv[2] * k * d[2]
    u0 = np.cos(phase)
    um1 = np.cos(phase + omega * dt)
    nt = 200
    _, up, u = ora.forward(v, nt, dt, d=d, periodic=True, state=(um1, u0))
    assert np.abs(u - np.cos(phase - omega * nt * dt)).max() < 1e-10
    assert np.abs(up - np.cos(phase - omega * (nt - 1) * dt)).max() < 1e-10
    # the dispersion is real: at 3.3 points per z-wavelength the phase speed is off v
    assert omega / np.sqrt(sum(x * x for x in kv)) != pytest.approx(v0, rel=1e-3)


def test_stability_limit(ora):
    """The checkerboard mode has the largest symbol; leapfrog stays bounded iff
    v dt sqrt(K_max) <= 2, i.e. Courant <= 2/sqrt(3 s(pi)) = 0.45286 on a cube."""
    c = derived_weights()
    cstar = 2.0 / np.sqrt(3.0 * symbol(np.pi, c))
    assert abs(cstar - 0.452858) < 1e-5
    n = 8
    v = np.full((n, n, n), 2000.0, dtype=np.float32)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    chk = (-1.0) ** (i + j + k)
    amp = {}
    for cour in (0.99 * cstar, 1.01 * cstar):
        dt = ora.cfl_dt(v, 10.0, courant=cour)
        _, _, u = ora.forward(v, 400, dt, periodic=True, state=(chk, chk))
        amp[cour] = np.abs(u).max()
    assert amp[0.99 * cstar] < 20.0
    assert amp[1.01 * cstar] > 1e3


@pytest.mark.parametrize("periodic", [False, True])
def test_energy_conserved_without_sponge(ora, periodic):
    nx, ny, nz = 14, 12, 16
    d = (10.0, 10.0, 10.0)
    v = layered_velocity(nx, ny, nz, seed=1)
    dt = ora.cfl_dt(v, 10.0)
    q = ora.vdt2(v, dt)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u0 = np.exp(-((i - 7) ** 2 + (j - 6) ** 2 + (k - 8) ** 2) / 6.0)
    state = (u0, u0)
    E = []
    for n in range(60):
        _, up, u = ora.forward(v, 1, dt, d=d, periodic=periodic, state=state)
        E.append(energy(ora, state[0], state[1], u, q, d, periodic))
        state = (up, u)
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-12 * abs(E[0])


def test_sponge_dissipation_identity(ora):
    """I^n - I^{n-1} = -sum eta (u^{n+1} - u^{n-1})^2 / q exactly."""
    nx, ny, nz = 20, 18, 16
    d = (10.0, 10.0, 10.0)
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=2.0)
    dt = ora.cfl_dt(v, 10.0)
    q = ora.vdt2(v, dt)
    eta = ora.sponge_tables(nx, ny, nz, 5, float(v.max()), d, dt)
    etaf = eta[2][:, None, None] + eta[1][None, :, None] + eta[0][None, None, :]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u0 = np.exp(-((i - 10) ** 2 + (j - 9) ** 2 + (k - 8) ** 2) / 5.0)
    state = (np.zeros_like(u0), u0)
    prevI = None
    worst = 0.0
    for n in range(80):
        _, up, u = ora.forward(v, 1, dt, d=d, eta=eta, state=state)
        In = energy(ora, state[0], state[1], u, q, d, False)
        if prevI is not None:
            loss = -np.sum(etaf * (u - state[0]) ** 2 / q)
            worst = max(worst, abs((In - prevI) - loss) / abs(prevI))
        prevI = In
        state = (up, u)
    assert worst <= 1e-12
    assert prevI < 0.7 * energy(ora, np.zeros_like(u0), u0, *ora.forward(
        v, 1, dt, d=d, eta=eta, state=(np.zeros_like(u0), u0))[2:], q, d, False)


def test_reciprocity_with_sponge(ora):
    nx, ny, nz = 22, 20, 18
    d = (10.0, 9.0, 11.0)
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=2.0)
    dt = ora.cfl_dt(v, min(d))
    eta = ora.sponge_tables(nx, ny, nz, 4, float(v.max()), d, dt)
    w = ora.ricker(120, dt)
    s = (2, 7, 5)  # inside the sponge: its injection weight 1/(1+eta) matters
    r = (15, 12, 13)
    tr_sr, _, _ = ora.forward(v, 120, dt, d=d, src=s, w=w, eta=eta,
                              rec=np.array([r], np.int32))
    tr_rs, _, _ = ora.forward(v, 120, dt, d=d, src=r, w=w, eta=eta,
                              rec=np.array([s], np.int32))
    assert np.abs(tr_sr).max() > 1e-6
    assert np.abs(tr_sr - tr_rs).max() <= 1e-12 * np.abs(tr_sr).max()


def test_linearity_in_the_wavelet(ora):
    nx = ny = nz = 12
    v = layered_velocity(nx, ny, nz)
    dt = ora.cfl_dt(v, 10.0)
    w1 = ora.ricker(30, dt)
    w2 = np.sin(np.arange(30) * 0.3)
    rec = np.array([[3, 4, 5], [8, 8, 8]], np.int32)
    t1 = ora.forward(v, 30, dt, src=(6, 6, 6), w=w1, rec=rec)[0]
    t2 = ora.forward(v, 30, dt, src=(6, 6, 6), w=w2, rec=rec)[0]
    t12 = ora.forward(v, 30, dt, src=(6, 6, 6), w=2.0 * w1 - 3.0 * w2, rec=rec)[0]
    assert np.abs(t12 - (2 * t1 - 3 * t2)).max() <= 1e-12 * np.abs(t12).max()


def test_mirror_symmetry_bitwise(ora):
    n = 21
    a = smooth_velocity(n, n, n, seed=7, sigma=2.0).astype(np.float64)
    for ax in range(3):
        a = 0.5 * (a + np.flip(a, axis=ax))
    v = a.astype(np.float32)
    dt = ora.cfl_dt(v, 10.0)
    eta = ora.sponge_tables(n, n, n, 4, float(v.max()), (10.0,) * 3, dt)
    w = ora.ricker(40, dt)
    _, _, u = ora.forward(v, 40, dt, src=(10, 10, 10), w=w, eta=eta)
    assert np.abs(u).max() > 0
    for ax in range(3):
        assert same_bits(u, np.flip(u, axis=ax))


def test_resume_is_bitwise(ora):
    nx, ny, nz = 16, 14, 12
    v = layered_velocity(nx, ny, nz)
    dt = ora.cfl_dt(v, 10.0)
    eta = ora.sponge_tables(nx, ny, nz, 3, float(v.max()), (10.0,) * 3, dt)
    w = ora.ricker(100, dt)
    rec = np.array([[1, 2, 3], [8, 7, 6]], np.int32)
    t_all, up_all, u_all = ora.forward(v, 100, dt, src=(8, 7, 6), w=w, eta=eta, rec=rec)
    t_a, up_a, u_a = ora.forward(v, 50, dt, src=(8, 7, 6), w=w[:50], eta=eta, rec=rec)
    t_b, up_b, u_b = ora.forward(v, 50, dt, src=(8, 7, 6), w=w[50:], eta=eta, rec=rec,
                                 state=(up_a, u_a))
    assert same_bits(np.vstack([t_a, t_b]), t_all)
    assert same_bits(u_b, u_all) and same_bits(up_b, up_all)


# ----------------------------------------------------------------- source and sponge

def test_ricker_closed_form_properties(ora):
    f0 = 15.0
    t0 = 1.0 / f0
    dt = t0 / 10
    w = ora.ricker(21, dt, f0=f0, t0=t0)
    assert abs(w[10] - 1.0) < 1e-12
    assert np.all(w <= 1.0 + 1e-12)
    tz = 1.0 / (np.sqrt(2.0) * np.pi * f0)
    for t in (t0 - tz, t0 + tz):
        assert abs(ora.ricker(1, t, f0=f0, t0=t0, n0=1)[0]) < 1e-12
    # zero mean and spectral peak at f0 (the spectrum is prop. to f^2 exp(-f^2/f0^2))
    fine = 1e-4
    n0 = -int(round(0.5 / fine))
    ww = ora.ricker(int(round(1.0 / fine)), fine, f0=f0, t0=t0, n0=n0)
    assert abs(ww.sum() * fine) < 1e-10
    spec = np.abs(np.fft.rfft(ww, n=1 << 20))
    f = np.fft.rfftfreq(1 << 20, d=fine)
    assert abs(f[np.argmax(spec)] - f0) < 2 * (f[1] - f[0])
    # the first sample of the production delay t0 = 1/f0
    assert abs(ora.ricker(1, dt, f0=f0)[0] - (1 - 2 * np.pi ** 2) * np.exp(-np.pi ** 2)) < 1e-15


def test_sponge_profile_closed_form(ora):
    n, W = 64, 16
    vmax, d = 4500.0, 10.0
    dt = 0.4 * d / vmax
    eta = ora.sponge_eta(n, W, vmax, d, dt)
    # quadratic in the W outer cells of each side, zero inside, symmetric
    assert np.all(eta[W:n - W] == 0.0)
    assert np.all(eta[:W] > 0) and np.all(eta[n - W:] > 0)
    assert np.array_equal(eta, eta[::-1])
    i = np.arange(W)
    assert np.allclose(eta[:W] / eta[0], ((W - i) / W) ** 2, rtol=1e-14, atol=0)
    # a quadratic sigma of peak s over L = W d reflects exp(-2 s L / (3 v)) at normal
    # incidence; the peak is chosen so that this equals R = 1e-3
    smax = 2 * eta[0] / dt
    assert abs(np.exp(-2 * smax * W * d / (3 * vmax)) - 1e-3) < 1e-15
    # at Courant 0.4 the peak eta is 3 ln(1000) * 0.4 / 64, whatever v and d are
    assert abs(eta[0] - 3 * np.log(1000) * 0.4 / 64) < 1e-15
    assert np.all(ora.sponge_eta(n, 0, vmax, d, dt) == 0.0)


@pytest.mark.parametrize("periodic", [False, True])
def test_step_points_equals_one_full_step(ora, periodic):
    """The point-sampled step (used for full-size sampled parity) reproduces a whole
    oracle step exactly, including wrapped or zero neighbours and the source, on a
    grid with three different spacings."""
    nx, ny, nz = 15, 11, 9
    d = (10.0, 12.5, 8.0)
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=2.0)
    dt = ora.cfl_dt(v, min(d))
    eta = ora.sponge_tables(nx, ny, nz, 3, float(v.max()), d, dt)
    up = random_field((nz, ny, nx), 1)
    u = random_field((nz, ny, nx), 2)
    src = (3, 4, 5)
    w = np.array([0.7])
    _, _, full = ora.forward(v, 1, dt, d=d, src=src, w=w, eta=eta, periodic=periodic,
                             state=(up.astype(np.float64), u.astype(np.float64)))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.int32)
    got = ora.step_points(up, u, ora.vdt2(v, dt), pts, d=d, eta=eta, periodic=periodic,
                          src=src, w_src=0.7).reshape(full.shape)
    assert np.array_equal(got, full)
