"""Pins of the FP64 direct-sum oracle against what the physics fixes.

The oracle evaluates the half-space representation (paper Sec. 3, eq.
(v_sum_halfspace) and eq. (phi)).  Nothing here re-types those formulas; each
test checks a property that the true half-space Green's functions must have:

* no-slip on the wall x3 = 0 (Sec. 3: the image and Papkovich-Neuber terms are
  added exactly to enforce it),
* a divergence-free field and a Stokes flow (harmonic vorticity),
* harmonic correction potentials whose gradient is the one used,
* Lorentz reciprocity of the half-space stokeslet,
* a point force on the wall produces no flow,
* far from the wall the half-space sum tends to the free-space one (Sec. 2),
* linearity, self exclusion (Sec. 2, p != m), symmetry of the stresslet in
  (g, q), dependence of the rotlet on g x q only, and in-plane translation
  invariance without x3 invariance (Sec. 3).

Together no-slip, incompressibility, the Stokes equations, decay and the free
singularities determine the half-space field uniquely, so these pins fix every
term.  ``test_pins_catch_planted_mistakes`` plants mistakes in the oracle and
checks that each is caught.
"""
import numpy as np
import pytest

import oracle

KERNELS = ["stokeslet", "stresslet", "rotlet"]


def _strengths(kernel, n, g):
    if kernel == "stokeslet":
        return g.standard_normal((n, 3))
    return g.standard_normal((n, 6))


def _sources(n, g, zmin=0.2, zmax=1.0):
    y = g.random((n, 3))
    y[:, 2] = zmin + (zmax - zmin) * g.random(n)
    return y


def _far_targets(y, n, g, dmin, box=(-0.5, 1.5), zr=(0.0, 1.5)):
    out = []
    while len(out) < n:
        x = np.array([g.uniform(*box), g.uniform(*box), g.uniform(*zr)])
        if np.min(np.linalg.norm(y - x, axis=1)) > dmin and np.min(
            np.linalg.norm(y * [1, 1, -1] - x, axis=1)) > dmin:
            out.append(x)
    return np.array(out)


def _jacobian(kernel, y, s, x, h=1e-3):
    """du_i/dx_j by 4th-order central differences, shape (T, 3, 3)."""
    T = x.shape[0]
    J = np.zeros((T, 3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        pts = np.concatenate([x + 2 * e, x + e, x - e, x - 2 * e])
        u = oracle.halfspace(kernel, y, s, pts).reshape(4, T, 3)
        J[:, :, j] = (-u[0] + 8 * u[1] - 8 * u[2] + u[3]) / (12 * h)
    return J


def _laplacian(fun, x, h):
    """4th-order 13-point (per axis 5-point) Laplacian of a vector field fun(pts)->(P, k)."""
    T = x.shape[0]
    c = fun(x)
    acc = -3 * 30 * c
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        for off, w in ((2, -1), (1, 16), (-1, 16), (-2, -1)):
            acc = acc + w * fun(x + off * e)
    return acc / (12 * h * h)


@pytest.mark.parametrize("kernel", KERNELS)
def test_no_slip_on_wall(kernel):
    g = np.random.default_rng(11)
    y = _sources(40, g, zmin=0.01)
    s = _strengths(kernel, 40, g)
    x = g.random((64, 3)) * 2 - 0.5
    x[:, 2] = 0.0
    u = oracle.halfspace(kernel, y, s, x)
    x_off = x.copy()
    x_off[:, 2] = 0.25
    scale = np.sqrt(np.mean(oracle.halfspace(kernel, y, s, x_off) ** 2))
    assert np.max(np.abs(u)) <= 1e-13 * scale


@pytest.mark.parametrize("kernel", KERNELS)
def test_divergence_free(kernel):
    g = np.random.default_rng(12)
    y = _sources(6, g)
    s = _strengths(kernel, 6, g)
    x = _far_targets(y, 20, g, dmin=0.3)
    J = _jacobian(kernel, y, s, x)
    div = np.trace(J, axis1=1, axis2=2)
    scale = np.sqrt(np.mean(J**2))
    assert np.max(np.abs(div)) <= 1e-7 * scale


@pytest.mark.parametrize("kernel", KERNELS)
def test_stokes_flow_vorticity_is_harmonic(kernel):
    """Stokes equations: lap u = grad p, hence curl(lap u) = 0."""
    g = np.random.default_rng(13)
    y = _sources(5, g)
    s = _strengths(kernel, 5, g)
    x = _far_targets(y, 12, g, dmin=0.4)
    h = 1e-2

    def lap_u(p):
        return _laplacian(lambda q: oracle.halfspace(kernel, y, s, q), p, h)

    d = 2e-3
    curl = np.zeros((x.shape[0], 3))
    grads = []
    for j in range(3):
        e = np.zeros(3)
        e[j] = d
        # 4th-order d(lap u)/dx_j
        grads.append((-lap_u(x + 2 * e) + 8 * lap_u(x + e) - 8 * lap_u(x - e) + lap_u(x - 2 * e)) / (12 * d))
    # curl_i = eps_ijk d_j (lap u)_k
    curl[:, 0] = grads[1][:, 2] - grads[2][:, 1]
    curl[:, 1] = grads[2][:, 0] - grads[0][:, 2]
    curl[:, 2] = grads[0][:, 1] - grads[1][:, 0]
    scale = np.sqrt(np.mean(np.concatenate(grads) ** 2))
    assert np.max(np.abs(curl)) <= 1e-4 * scale


@pytest.mark.parametrize("kernel", KERNELS)
def test_correction_potential_harmonic_and_gradient(kernel):
    g = np.random.default_rng(14)
    y = _sources(1, g)
    s = _strengths(kernel, 1, g)
    h = 1e-3
    for x in _far_targets(y, 8, g, dmin=0.3):
        phi0, gphi = oracle.correction(kernel, y, s, x[None])
        fd = np.zeros(3)
        lap = -90.0 * phi0
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            vals = {k: oracle.correction(kernel, y, s, (x + k * e)[None])[0] for k in (2, 1, -1, -2)}
            fd[j] = (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)
            lap += -vals[2] + 16 * vals[1] + 16 * vals[-1] - vals[-2]
        lap /= 12 * h * h
        scale = np.linalg.norm(gphi) + abs(phi0)
        assert np.linalg.norm(fd - gphi) <= 1e-8 * scale
        assert abs(lap) <= 1e-4 * scale


def test_stokeslet_reciprocity():
    """G_ij(x, y) = G_ji(y, x) for the no-slip half-space Green's function."""
    g = np.random.default_rng(15)
    for _ in range(10):
        a = np.array([g.random(), g.random(), 0.05 + g.random()])
        b = np.array([g.random(), g.random(), 0.05 + g.random()])
        Gab = np.stack([oracle.halfspace("stokeslet", b[None], np.eye(3)[j][None], a[None])[0] for j in range(3)],
                       axis=1)
        Gba = np.stack([oracle.halfspace("stokeslet", a[None], np.eye(3)[j][None], b[None])[0] for j in range(3)],
                       axis=1)
        assert np.max(np.abs(Gab - Gba.T)) <= 1e-13 * np.max(np.abs(Gab))


def test_point_force_on_wall_gives_no_flow():
    g = np.random.default_rng(16)
    y = np.array([[0.4, 0.6, 1e-9]])
    f = g.standard_normal((1, 3))
    x = g.random((32, 3))
    x[:, 2] += 0.1
    u = oracle.halfspace("stokeslet", y, f, x)
    free = oracle.freespace("stokeslet", y, f, x)
    assert np.max(np.abs(u)) <= 1e-7 * np.max(np.abs(free))


@pytest.mark.parametrize("kernel", KERNELS)
def test_far_from_wall_tends_to_free_space(kernel):
    g = np.random.default_rng(17)
    s = _strengths(kernel, 1, g)
    errs = []
    for H in (1e2, 1e3, 1e4):
        y = np.array([[0.0, 0.0, H]])
        x = np.array([[0.7, -0.4, H + 0.3]])
        hs = oracle.halfspace(kernel, y, s, x)
        fs = oracle.freespace(kernel, y, s, x)
        errs.append(np.linalg.norm(hs - fs) / np.linalg.norm(fs))
    # the wall's influence decays at least like 1/H
    assert errs[2] < 2e-3 and errs[2] < errs[1] < errs[0]
    assert errs[1] / errs[2] > 5.0


@pytest.mark.parametrize("kernel", KERNELS)
def test_linearity_and_zero_strength(kernel):
    g = np.random.default_rng(18)
    y = _sources(30, g, zmin=0.01)
    x = g.random((25, 3))
    if kernel == "stokeslet":
        s1, s2 = g.standard_normal((30, 3)), g.standard_normal((30, 3))
        a, b = 0.7, -1.3
        u = oracle.halfspace(kernel, y, a * s1 + b * s2, x)
        ref = a * oracle.halfspace(kernel, y, s1, x) + b * oracle.halfspace(kernel, y, s2, x)
        assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.all(oracle.halfspace(kernel, y, 0 * s1, x) == 0.0)
    else:
        gq = g.standard_normal((30, 6))
        gq2 = gq.copy()
        gq2[:, :3] *= 2.5  # linear in the strength g
        u1 = oracle.halfspace(kernel, y, gq, x)
        u2 = oracle.halfspace(kernel, y, gq2, x)
        assert np.max(np.abs(u2 - 2.5 * u1)) <= 1e-12 * np.max(np.abs(u2))
        z = gq.copy()
        z[:, :3] = 0
        assert np.all(oracle.halfspace(kernel, y, z, x) == 0.0)


@pytest.mark.parametrize("kernel", KERNELS)
def test_self_exclusion_is_superposition(kernel):
    """u at a source point = sum over the other sources + own image/correction."""
    g = np.random.default_rng(19)
    y = _sources(12, g, zmin=0.01)
    s = _strengths(kernel, 12, g)
    u = oracle.halfspace(kernel, y, s, y)
    for p in range(12):
        others = np.delete(np.arange(12), p)
        ref = oracle.halfspace(kernel, y[others], s[others], y[p:p + 1])[0]
        own = oracle.halfspace(kernel, y[p:p + 1], s[p:p + 1], y[p:p + 1])[0]
        assert np.all(np.isfinite(own))
        assert np.max(np.abs(u[p] - ref - own)) <= 1e-12 * np.max(np.abs(u[p]))


def test_rotlet_depends_on_torque_only():
    g = np.random.default_rng(20)
    y = _sources(20, g, zmin=0.01)
    gq = g.standard_normal((20, 6))
    v = np.cross(gq[:, :3], gq[:, 3:])
    x = g.random((15, 3))
    u1 = oracle.halfspace("rotlet", y, gq, x)
    u2 = oracle.halfspace("rotlet", y, oracle.torque_to_pair(v), x)
    u3 = oracle.halfspace("rotlet", y, v, x)
    assert np.max(np.abs(u1 - u2)) <= 1e-12 * np.max(np.abs(u1))
    assert np.max(np.abs(u1 - u3)) <= 1e-12 * np.max(np.abs(u1))


def test_stresslet_symmetric_in_strength_and_orientation():
    g = np.random.default_rng(21)
    y = _sources(20, g, zmin=0.01)
    gq = g.standard_normal((20, 6))
    qg = np.concatenate([gq[:, 3:], gq[:, :3]], axis=1)
    x = g.random((15, 3))
    u1 = oracle.halfspace("stresslet", y, gq, x)
    u2 = oracle.halfspace("stresslet", y, qg, x)
    assert np.max(np.abs(u1 - u2)) <= 1e-12 * np.max(np.abs(u1))


@pytest.mark.parametrize("kernel", KERNELS)
def test_in_plane_translation_invariance_only(kernel):
    g = np.random.default_rng(22)
    y = _sources(20, g, zmin=0.01)
    s = _strengths(kernel, 20, g)
    x = g.random((15, 3))
    u = oracle.halfspace(kernel, y, s, x)
    d = np.array([0.37, -1.21, 0.0])
    u_shift = oracle.halfspace(kernel, y + d, s, x + d)
    assert np.max(np.abs(u - u_shift)) <= 1e-11 * np.max(np.abs(u))
    d3 = np.array([0.0, 0.0, 0.3])
    u_up = oracle.halfspace(kernel, y + d3, s, x + d3)
    assert np.max(np.abs(u - u_up)) > 1e-3 * np.max(np.abs(u))


def test_pins_catch_planted_mistakes():
    """Each planted mistake in the oracle breaks no-slip or incompressibility."""
    g = np.random.default_rng(23)
    y = _sources(6, g)
    wall = g.random((16, 3))
    wall[:, 2] = 0.0
    kernels_for = {1: "stokeslet", 2: "stresslet", 3: "stokeslet", 4: "rotlet"}
    try:
        for m, kernel in kernels_for.items():
            s = _strengths(kernel, 6, g)
            oracle.set_mutation(m)
            u_wall = oracle.halfspace(kernel, y, s, wall)
            x = _far_targets(y, 10, g, dmin=0.3)
            J = _jacobian(kernel, y, s, x)
            div = np.max(np.abs(np.trace(J, axis1=1, axis2=2))) / np.sqrt(np.mean(J**2))
            off = wall.copy()
            off[:, 2] = 0.25
            scale = np.sqrt(np.mean(oracle.halfspace(kernel, y, s, off) ** 2))
            slip = np.max(np.abs(u_wall)) / scale
            assert slip > 1e-3 or div > 1e-3, f"mutation {m} not caught (slip {slip}, div {div})"
    finally:
        oracle.set_mutation(0)


# ---------------------------------------------------------------------------
# The real-space part of the Ewald split (oracle.ewald_real): the kernels of
# the appendix's eq. (kernel_real_parts) and the corrections with
# G_R = erfc(xi r)/r of eq. (G_R).  Pinned by two limits that the paper fixes:
#   * xi -> 0 with every pair inside r_c: the real part is the whole sum
#     (erfc -> 1, the Gaussian terms vanish), so it tends to the direct sum
#     at rate xi (stokeslet: its self and Gaussian terms) or faster;
#   * r -> 0 at fixed xi: K_R - K and the corrections with G_R minus those
#     with G stay finite, with limits from the Taylor series of erf
#     (Sec. 4: the stokeslet's self term -4 xi/sqrt(pi) f is the first), so
#     every Gaussian term's coefficient, which cancels a singular part of the
#     erfc term, is fixed; a wrong one leaves a term of order 1/r or worse.
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("kernel", KERNELS)
def test_real_part_tends_to_the_whole_sum_as_xi_vanishes(kernel):
    g = np.random.default_rng(17)
    y, s = _sources(60, g), _strengths(kernel, 60, g)
    full = oracle.halfspace(kernel, y, s, y)
    scale = np.sqrt(np.mean(full ** 2))
    errs = []
    for xi in (1e-6, 1e-4):
        re = oracle.ewald_real(kernel, y, s, y, xi, 1e9)
        errs.append(np.sqrt(np.mean((re - full) ** 2)) / scale)
    print(kernel, errs)
    if kernel == "stokeslet":
        # linear in xi: the ratio of the two errors is the ratio of the xi
        assert 50 < errs[1] / errs[0] < 200
        assert errs[1] < 1e-3
    else:
        assert max(errs) < 1e-12


def _direct_limit_err(kernel, delta, xi=7.0):
    """|(K_R - K)(delta n) s - its expansion at r -> 0|, relative, for one
    source (r_c excludes the image) and a random direction n.

    K_R - K = -K_F, and K_F is smooth, so the expansion is -K_F(0) -
    r.grad K_F(0) + O(r^2), taken from the Fourier multipliers of the
    appendix, not from the real-space formulas.  The stokeslet's K_F(0) is
    minus the self term of Sec. 4.  The stresslet's and the rotlet's are odd,
    so K_F(0) = 0, and the angular averages <k_n k_m> = k^2 delta_nm / 3 and
    <k_n k_j k_l k_m> = k^4 (sym. deltas) / 15 reduce grad K_F(0) to one
    radial integral: with B^ = -8 pi/k^4 (biharmonic) and H^ = 4 pi/k^2
    (harmonic), d_n T_F,jlm(0) = -(4 xi^3/sqrt(pi))(d_nm d_jl + d_nj d_lm +
    d_nl d_mj) and d_n W_F,jl(0) = (8 xi^3/(3 sqrt(pi))) eps_jln (the rotlet
    multiplier with the sign fixed by W = 2 eps r / r^3)."""
    c = 2.0 * xi / np.sqrt(np.pi)
    g = np.random.default_rng(23)
    y = np.array([[0.3, 0.4, 0.6]])
    s = g.standard_normal((1, 3 if kernel == "stokeslet" else 6))
    n = g.standard_normal(3)
    n /= np.linalg.norm(n)
    x = y + delta * n
    d = oracle.ewald_real(kernel, y, s, x, xi, 0.5)[0] - oracle.freespace(kernel, y, s, x)[0]
    if kernel == "stokeslet":
        lim = -2.0 * c * s[0]  # -4 xi/sqrt(pi) f, the self term of Sec. 4
    elif kernel == "stresslet":
        gv, qv = s[0, :3], s[0, 3:]
        lim = 4.0 * xi ** 3 / np.sqrt(np.pi) * delta * (gv * (n @ qv) + (gv @ qv) * n + qv * (n @ gv))
    else:
        v = np.cross(s[0, :3], s[0, 3:])
        lim = -8.0 * xi ** 3 / (3.0 * np.sqrt(np.pi)) * delta * np.cross(v, n)
    return np.linalg.norm(d - lim) / max(1.0, np.linalg.norm(lim))


def _correction_limit_err(kernel, delta, xi=5.0):
    """H = G_R - G = -erf(xi r)/r has H(0) = -c, grad H(0) = 0,
    grad grad H(0) = (2/3) c xi^2 I and zero third derivatives (c =
    2 xi/sqrt(pi)), so at r~ = x - y^I -> 0 the corrections with G_R and with
    G differ by closed forms; returns the relative errors of phi and grad phi."""
    c = 2.0 * xi / np.sqrt(np.pi)
    h2 = 2.0 * c * xi ** 2 / 3.0
    g = np.random.default_rng(29)
    y = np.array([[0.2, 0.7, 0.35]])
    s = g.standard_normal((1, 3 if kernel == "stokeslet" else 6))
    ss, y3 = s[0], y[0, 2]
    n = g.standard_normal(3)
    n /= np.linalg.norm(n)
    x = (y[0] * np.array([1.0, 1.0, -1.0]) + delta * n)[None, :]
    p_r, g_r = oracle.correction_real(kernel, y, s, x, xi)
    p_0, g_0 = oracle.correction(kernel, y, s, x)
    flip = np.array([1.0, 1.0, -1.0])
    if kernel == "stokeslet":
        lp, lg = 2.0 * c * ss[2], -2.0 * y3 * h2 * ss * flip
    elif kernel == "stresslet":
        gI, qI = ss[:3] * flip, ss[3:] * flip
        lp, lg = -4.0 * y3 * h2 * (gI @ qI), 4.0 * (gI @ qI) * h2 * np.array([0.0, 0.0, 1.0])
    else:
        gI, qI = ss[:3] * flip, ss[3:] * flip
        lp, lg = 0.0, 2.0 * h2 * 2.0 * (ss[5] * gI - ss[2] * qI)
    return (abs((p_r - p_0) - lp) / max(1.0, abs(lp)),
            np.linalg.norm((g_r - g_0) - lg) / max(1.0, np.linalg.norm(lg)))


def _real_correction_gradient_err(kernel, xi=5.0):
    """grad phi_R against 4th-order differences of phi_R (both with G_R):
    ties the first three r-derivatives of G_R to G_R = erfc(xi r)/r itself."""
    g = np.random.default_rng(31)
    y = _sources(1, g)
    s = _strengths(kernel, 1, g)
    h, worst = 1e-4, 0.0
    for k in range(6):
        n = g.standard_normal(3)
        n /= np.linalg.norm(n)
        x = y[0] * np.array([1.0, 1.0, -1.0]) + (0.05 + 0.06 * k) * n
        _, gphi = oracle.correction_real(kernel, y, s, x[None], xi)
        fd = np.zeros(3)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            v = {m: oracle.correction_real(kernel, y, s, (x + m * e)[None], xi)[0] for m in (2, 1, -1, -2)}
            fd[j] = (-v[2] + 8 * v[1] - 8 * v[-1] + v[-2]) / (12 * h)
        worst = max(worst, np.linalg.norm(fd - gphi) / max(1.0, np.linalg.norm(gphi)))
    return worst


def _converges(err, d):
    """The error against a limit taken at distance d and d/10: a wrong
    constant or a dropped term that does not vanish as r -> 0 leaves it
    (nearly) unchanged; the right one falls at least tenfold per decade
    when it is first order, and to well below the size of the limit."""
    e1, e2 = err(d), err(d / 10)
    return e2 <= e1 / 5 and e2 < 5e-2, (e1, e2)


@pytest.mark.parametrize("kernel", KERNELS)
def test_real_kernels_minus_kernels_at_zero_distance(kernel):
    ok, e = _converges(lambda d: _direct_limit_err(kernel, d), 1e-3)
    print(kernel, e)
    assert ok


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("part", [0, 1])
def test_real_corrections_minus_corrections_at_zero_distance(kernel, part):
    # d from 1e-2 down to 1e-3: below ~3e-4 the cancellation in the third
    # derivatives of G_R (terms of size 1/r^4) reaches the truncation error
    ok, e = _converges(lambda d: _correction_limit_err(kernel, d)[part], 1e-2)
    print(kernel, part, e)
    assert ok


@pytest.mark.parametrize("kernel", KERNELS)
def test_real_correction_gradient_is_the_gradient_of_its_potential(kernel):
    err = _real_correction_gradient_err(kernel)
    print(kernel, err)
    assert err < 1e-7


@pytest.mark.parametrize("kernel", KERNELS)
def test_real_part_scales_with_the_kernel(kernel):
    """K_R depends on r only through xi r and carries the dimension of K
    (1/length for the stokeslet, 1/length^2 for the stresslet and rotlet),
    and so do the corrections built from G_R: scaling every position and r_c
    by lam and xi by 1/lam scales the real-space part by lam^-1 or lam^-2."""
    print(kernel, _scaling_err(kernel))
    assert _scaling_err(kernel) < 1e-12


def _scaling_err(kernel):
    g = np.random.default_rng(37)
    y = _sources(40, g)
    s = _strengths(kernel, 40, g)
    x = _sources(30, g)
    xi, rc, lam = 6.0, 0.35, 2.5
    d = 1 if kernel == "stokeslet" else 2
    u1 = oracle.ewald_real(kernel, y, s, x, xi, rc)
    u2 = oracle.ewald_real(kernel, lam * y, s, lam * x, xi / lam, lam * rc)
    return np.linalg.norm(u2 * lam ** d - u1) / np.linalg.norm(u1)


def test_split_pins_catch_planted_mistakes():
    """A wrong Gaussian coefficient in S_R (5), T_R (6) or W_R (7), a
    dropped term of the second (8) or third (9) r-derivative of G_R, or unit
    vectors in the Gaussian term of T_R (10) fail the pins above."""
    checks = {
        5: lambda: not _converges(lambda d: _direct_limit_err("stokeslet", d), 1e-3)[0],
        6: lambda: not _converges(lambda d: _direct_limit_err("stresslet", d), 1e-3)[0],
        7: lambda: not _converges(lambda d: _direct_limit_err("rotlet", d), 1e-3)[0],
        8: lambda: not _converges(lambda d: _correction_limit_err("stokeslet", d)[1], 1e-2)[0],
        9: lambda: _real_correction_gradient_err("stresslet") > 1e-7,
        10: lambda: (_scaling_err("stresslet") > 1e-12
                     and not _converges(lambda d: _direct_limit_err("stresslet", d), 1e-3)[0]),
    }
    try:
        for m, caught in checks.items():
            oracle.set_mutation(m)
            assert caught(), f"mutation {m} not caught"
    finally:
        oracle.set_mutation(0)
