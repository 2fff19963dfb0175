"""Pins of the oracle's adjoint step and FWI gradient (FP64).

The gradient with respect to squared slowness m = 1/v^2 is the exact transpose of the
forward recurrence; it is pinned by dot-product tests (the transpose identity
<F x, y> = <x, F^T y>, which a wrong sign, index or dropped term breaks), by the exact
linearity of one step in vdt2, and by central finite differences of the misfit.
"""
import numpy as np
import pytest

from workloads import blob_perturbed, random_field, receivers_plane, smooth_velocity

D = (10.0, 10.0, 10.0)


def _setup(ora, nx, ny, nz, W=4, seed=2):
    v = smooth_velocity(nx, ny, nz, seed=seed, sigma=2.0)
    dt = ora.cfl_dt(v, 10.0)
    q = ora.vdt2(v, dt)
    eta = ora.sponge_tables(nx, ny, nz, W, float(v.max()), D, dt)
    return v, dt, q, eta


def _step(ora, x1, x2, q, eta, periodic):
    b1, b2 = ora.to_box(x1), ora.to_box(x2)
    if periodic:
        ora.fill_halo_periodic(b2)
    return ora.interior(ora.step_box(b1, b2, ora.to_box(q), D, eta)).copy()


@pytest.mark.parametrize("periodic", [False, True])
def test_one_step_dot_test(ora, periodic):
    nx, ny, nz = 13, 11, 12
    v, dt, q, eta = _setup(ora, nx, ny, nz)
    x1 = random_field((nz, ny, nx), 1, dtype=np.float64)
    x2 = random_field((nz, ny, nx), 2, dtype=np.float64)
    y = random_field((nz, ny, nx), 3, dtype=np.float64)
    lhs = np.sum(_step(ora, x1, x2, q, eta, periodic) * y)
    a2, _ = ora.adjoint_step(None, y, q, D, eta, periodic)        # d/dx2
    a1, _ = ora.adjoint_step(y, np.zeros_like(y), q, D, eta, periodic)  # d/dx1
    rhs = np.sum(x2 * a2) + np.sum(x1 * a1)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("src", [None, (2, 5, 4), (6, 5, 4)])
def test_one_step_gradient_part_is_exact_derivative_in_vdt2(ora, src):
    """One step (source included) is affine in vdt2, so <g, dq> must equal
    <y, F(q+dq) - F(q)>; also at the source voxel alone, in and out of the sponge."""
    nx, ny, nz = 12, 10, 9
    v, dt, q, eta = _setup(ora, nx, ny, nz)
    x1 = random_field((nz, ny, nx), 4, dtype=np.float64)
    x2 = random_field((nz, ny, nx), 5, dtype=np.float64)
    y = random_field((nz, ny, nx), 6, dtype=np.float64)
    w0 = 37.0

    def F(qq):
        if src is None:
            return ora.forward(None, 1, dt, eta=eta, state=(x1, x2), q=qq)[2]
        return ora.forward(None, 1, dt, eta=eta, state=(x1, x2), q=qq, src=src,
                           w=np.array([w0]))[2]

    _, g = ora.adjoint_step(None, y, q, D, eta, False, u_n=x2, g=np.zeros_like(y),
                            w=w0 if src else 0.0, src=src)
    dq = 1e-3 * q * random_field((nz, ny, nx), 7, dtype=np.float64)
    diff = F(q + dq) - F(q)
    assert abs(np.sum(g * dq) - np.sum(y * diff)) <= 1e-12 * abs(np.sum(y * diff))
    if src is not None:
        dq1 = np.zeros_like(q)
        dq1[src[2], src[1], src[0]] = 1e-3 * q[src[2], src[1], src[0]]
        diff1 = F(q + dq1) - F(q)
        assert abs(np.sum(g * dq1) - np.sum(y * diff1)) <= 1e-12 * abs(np.sum(y * diff1))


def test_multi_step_dot_test_wavelet_to_traces(ora):
    """F: wavelet -> traces is linear; grad_w of J with obs = F w - r is F^T r."""
    nx, ny, nz, nt = 14, 12, 13, 70
    v, dt, q, eta = _setup(ora, nx, ny, nz)
    src = (7, 6, 6)
    rec = receivers_plane(nx, ny, 3)
    w = ora.ricker(nt, dt)
    r = random_field((nt, rec.shape[0]), 8, dtype=np.float64)
    Fw = ora.forward(v, nt, dt, src=src, w=w, eta=eta, rec=rec)[0]
    res = ora.fwi_gradient(v, nt, dt, Fw - r, src, w, rec, D, eta)
    assert np.allclose(res["traces"], Fw, rtol=0, atol=1e-15 * np.abs(Fw).max())
    w2 = random_field((nt,), 9, dtype=np.float64)
    Fw2 = ora.forward(v, nt, dt, src=src, w=w2, eta=eta, rec=rec)[0]
    lhs = np.sum(Fw2 * r)
    rhs = np.sum(w2 * res["grad_w"])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fwi_gradient_matches_central_differences(ora):
    nx, ny, nz, nt = 18, 16, 17, 90
    v0, dt, q0, eta = _setup(ora, nx, ny, nz)
    src = (9, 8, 3)
    rec = receivers_plane(nx, ny, 3)
    w = ora.ricker(nt, dt, f0=40.0)
    vt = blob_perturbed(v0, center=(9, 8, 10), radius=3.0)
    obs = ora.forward(vt, nt, dt, src=src, w=w, eta=eta, rec=rec)[0]
    m0 = 1.0 / v0.astype(np.float64) ** 2
    res = ora.fwi_gradient(None, nt, dt, obs, src, w, rec, D, eta, q=dt * dt / m0)
    g = res["grad_m"]
    assert np.abs(g).max() > 0
    from workloads import fd_voxels
    vox = list(fd_voxels(g, count=8, seed=5))
    vox.append(np.ravel_multi_index((src[2], src[1], src[0]), g.shape))  # source voxel

    def J(m):
        tr = ora.forward(None, nt, dt, src=src, w=w, eta=eta, rec=rec, q=dt * dt / m)[0]
        return 0.5 * np.sum((tr - obs) ** 2)

    for p in vox:
        h = 1e-4 * m0.flat[p]
        mp = m0.copy()
        mp.flat[p] += h
        mm = m0.copy()
        mm.flat[p] -= h
        fd = (J(mp) - J(mm)) / (2 * h)
        assert abs(fd - g.flat[p]) <= 1e-6 * abs(g.flat[p]), (p, fd, g.flat[p])
