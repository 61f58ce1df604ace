"""Brute-force twin of the oracle at 50 significant digits, tiny N.

An independent evaluation of the half-space sum (paper Sec. 3, eq.
(v_sum_halfspace) with the correction potentials of eq. (phi)) in mpmath at
50 digits, written from the paper and not from the oracle's source:

* the free-space kernels are contracted index by index from their tensor
  definitions (Sec. 2, with the normalisation that makes the wall velocity
  vanish: S_ij = delta_ij/r + r_i r_j/r^3, T_ijk = -6 r_i r_j r_k/r^5 and
  the rotlet 2 (v x r)/r^3 with v = g x q);
* the image of each source is applied with its reflected strengths, the
  rotlet's image through g^I x q^I itself (not through the torque);
* every derivative of G = 1/|x - y^I| in phi, and the gradient of phi that
  enters -x_3 grad phi, is taken by mpmath's numerical differentiation at
  50 digits, not from closed forms as in the oracle;
* the stresslet correction is phi_T = 4 (g^I . q^I) d3 G - 4 y3 (g^I)^T
  (grad grad G) q^I (the harmonic function with the wall values that no-slip
  requires; the printed second coefficient does not give no-slip).

The oracle must agree element by element to FP64 rounding: targets at the
sources (their own direct term omitted, Sec. 2 p != m), targets on the wall
x3 = 0 and sources 1e-8 above the wall, where the direct, image and
correction terms cancel to many digits.
"""
import numpy as np
import pytest

import oracle

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp

KERNELS = ["stokeslet", "stresslet", "rotlet"]


def _m(v):
    return [mp.mpf(float(a)) for a in v]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _norm(r):
    return mp.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)


def _kernel(kernel, r, s):
    """Free-space kernel applied to strengths s at separation r (Sec. 2)."""
    rn = _norm(r)
    out = [mp.mpf(0)] * 3
    if kernel == "stokeslet":
        for i in range(3):
            for j in range(3):
                Sij = (1 if i == j else 0) / rn + r[i] * r[j] / rn**3
                out[i] += Sij * s[j]
    elif kernel == "stresslet":
        g, q = s[:3], s[3:]
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    out[i] += -6 * r[i] * r[j] * r[k] / rn**5 * g[j] * q[k]
    else:
        v = s
        eps = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}
        for (i, j, k), e in eps.items():
            out[i] += 2 * e * v[j] * r[k] / rn**3
    return out


def _G_derivs(x, yI):
    """G = 1/|x - y^I| and its first and second derivatives in x (numerical, 50 digits)."""

    def G(a, b, c):
        return 1 / mp.sqrt((a - yI[0]) ** 2 + (b - yI[1]) ** 2 + (c - yI[2]) ** 2)

    d1 = []
    for i in range(3):
        n = [0, 0, 0]
        n[i] = 1
        d1.append(mp.diff(G, x, tuple(n)))
    d2 = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            n = [0, 0, 0]
            n[i] += 1
            n[j] += 1
            d2[i][j] = mp.diff(G, x, tuple(n))
    return G(*x), d1, d2


def _phi(kernel, y, s, x):
    """Correction potential of one source at the point x (eq. (phi))."""
    yI = [y[0], y[1], -y[2]]
    G, dG, ddG = _G_derivs(x, yI)
    y3 = y[2]
    if kernel == "stokeslet":
        fI = [s[0], s[1], -s[2]]
        return 2 * (-s[2] * G - y3 * sum(dG[i] * fI[i] for i in range(3)))
    g, q = s[:3], s[3:]
    gI = [g[0], g[1], -g[2]]
    qI = [q[0], q[1], -q[2]]
    if kernel == "stresslet":
        gq = sum(gI[i] * qI[i] for i in range(3))
        quad = sum(gI[i] * ddG[i][j] * qI[j] for i in range(3) for j in range(3))
        return 4 * gq * dG[2] - 4 * y3 * quad
    w = [2 * (q[2] * gI[i] - g[2] * qI[i]) for i in range(3)]
    return 2 * sum(dG[i] * w[i] for i in range(3))


def twin(kernel, y, s, x):
    """u(x_t) = sum_m K(x - y_m) s_m - K(x - y_m^I) s_m^I - x3 grad phi_m + e3 phi_m, 50 digits."""
    out = np.zeros((len(x), 3))
    for t in range(len(x)):
        xt = _m(x[t])
        acc = [mp.mpf(0)] * 3
        for m in range(len(y)):
            ym = _m(y[m])
            sm = _m(s[m])
            r = [xt[i] - ym[i] for i in range(3)]
            if any(r):
                direct_s = sm if kernel != "rotlet" else _cross(sm[:3], sm[3:])
                k = _kernel(kernel, r, direct_s)
                acc = [acc[i] + k[i] for i in range(3)]
            rt = [xt[0] - ym[0], xt[1] - ym[1], xt[2] + ym[2]]
            if kernel == "stokeslet":
                img = _kernel(kernel, rt, [sm[0], sm[1], -sm[2]])
            elif kernel == "stresslet":
                img = _kernel(kernel, rt, [sm[0], sm[1], -sm[2], sm[3], sm[4], -sm[5]])
            else:
                gI = [sm[0], sm[1], -sm[2]]
                qI = [sm[3], sm[4], -sm[5]]
                img = _kernel(kernel, rt, _cross(gI, qI))
            acc = [acc[i] - img[i] for i in range(3)]

            def phi_at(a, b, c, ym=ym, sm=sm):
                return _phi(kernel, ym, sm, [a, b, c])

            ph = phi_at(*xt)
            gph = []
            for i in range(3):
                n = [0, 0, 0]
                n[i] = 1
                gph.append(mp.diff(phi_at, xt, tuple(n)))
            acc = [acc[0] - xt[2] * gph[0], acc[1] - xt[2] * gph[1], acc[2] - xt[2] * gph[2] + ph]
        out[t] = [float(a) for a in acc]
    return out


def _case(kernel, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    n = 12
    y = g.random((n, 3))
    y[:, 2] = 0.05 + 0.95 * y[:, 2]
    y[0, 2] = 1e-8   # sources just above the wall
    y[1, 2] = 3e-8
    y[2, 2] = 1e-3
    s = g.standard_normal((n, 3 if kernel == "stokeslet" else 6))
    wall = g.random((3, 3))
    wall[:, 2] = 0.0
    wall[0, :2] = y[0, :2]  # on the wall right below a near-wall source
    free = g.random((3, 3))
    x = np.concatenate([y, wall, free])  # the sources themselves, the wall, elsewhere
    return y, s, x


@pytest.mark.parametrize("kernel", KERNELS)
def test_oracle_matches_50_digit_twin(kernel):
    mp.dps = 50
    y, s, x = _case(kernel, 1802 + KERNELS.index(kernel))
    ref = twin(kernel, y, s, x)
    u = oracle.halfspace(kernel, y, s, x)
    rms = np.sqrt(np.mean(np.sum(ref**2, axis=1)))
    err = np.linalg.norm(u - ref, axis=1)
    scale = np.maximum(np.linalg.norm(ref, axis=1), rms)
    # per target, relative to its own velocity or the RMS velocity where that is
    # larger (wall targets): FP64 rounding only
    assert np.all(err <= 1e-14 * scale), (kernel, (err / scale).max())
    assert oracle.rel_rms(ref, u) <= 1e-14
    # the wall rows of the twin itself vanish (no-slip), so the twin is no copy of a broken formula
    nw = len(y)
    assert np.all(np.abs(ref[nw:nw + 3]) <= 1e-12 * rms)


def test_twin_catches_planted_oracle_mistakes():
    """Each planted oracle mistake moves it far outside the twin's bound."""
    mp.dps = 30
    for kernel, mut in (("stokeslet", 1), ("stresslet", 2), ("rotlet", 3), ("stokeslet", 4)):
        y, s, x = _case(kernel, 7)
        y, s, x = y[3:7], s[3:7], x[:6]
        ref = twin(kernel, y, s, x)
        try:
            oracle.set_mutation(mut)
            bad = oracle.halfspace(kernel, y, s, x)
        finally:
            oracle.set_mutation(0)
        assert oracle.rel_rms(ref, bad) > 1e-6, (kernel, mut)
