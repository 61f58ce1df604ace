"""Stage-level checks of the GPU path, so that a failure names its stage.

The real-space sum's cell lists (Sec. 4 and 5.1: pairs within r_c only) are
checked by count: the kernels count the (target, source) pairs they
evaluate (direct pairs with 0 < |x - y| < r_c, image pairs with
|x - y^I| < r_c, y^I = (y1, y2, -y3)), which must equal a brute-force count
over all pairs, for every cell reach and for point sets uniform and
clustered at the wall, with the targets the sources or separate.  A cell
walk that misses a neighbour cell, or visits one twice, changes the count.

The split of the sum into its real-space and Fourier parts (Sec. 4) is
checked part by part against the oracle's split, so that an error names the
half it sits in.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1802_07844_amd as ehs  # noqa: E402
from paper_1802_07844_amd import workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _brute_counts(y, x, rc):
    """Pairs with 0 < r^2 < r_c^2 and image pairs with r~^2 < r_c^2, by
    brute force over target blocks."""
    rc2 = rc * rc
    nd = ni = 0
    yi = y * np.array([1.0, 1.0, -1.0])
    for t0 in range(0, len(x), 512):
        xb = x[t0:t0 + 512]
        d = xb[:, None, :] - y[None, :, :]
        r2 = (d * d).sum(axis=2)
        nd += int(np.count_nonzero((r2 < rc2) & (r2 > 0.0)))
        d = xb[:, None, :] - yi[None, :, :]
        r2 = (d * d).sum(axis=2)
        ni += int(np.count_nonzero(r2 < rc2))
    return nd, ni


@pytest.mark.parametrize("layout", ["uniform", "clustered"])
@pytest.mark.parametrize("reach", [0, 1, 2, 3])
def test_pair_counts_match_brute_force(layout, reach):
    n, t = 8_000, 3_000
    g = workloads.rng(workloads.SEED_BASE + 70)
    y, f = workloads.make("stokeslet", n, workloads.SEED_BASE + 71, layout=layout)
    # separate targets from the same distribution, and coincident ones
    xs, _ = workloads.make("stokeslet", t, workloads.SEED_BASE + 72, layout=layout)
    xs[:50] = y[g.choice(n, 50, replace=False)]
    rc = 0.12 if layout == "uniform" else 0.06
    tol = 1e-10
    xi = ehs.xi_for_cutoff("stokeslet", rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        c.set_option(ehs.OPT_TIMING, 1)
        c.set_option(ehs.OPT_CELL_REACH, reach)
        yd, fd = torch.from_numpy(y).to(DEV), torch.from_numpy(f).to(DEV)
        for label, x in (("targets = sources", y), ("separate targets", xs)):
            xd = yd if x is y else torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
            u, rep = c.evaluate("stokeslet", yd, fd, xd, xi, rc, tol, report=True)
            torch.cuda.synchronize()
            nd, ni = _brute_counts(y, x, rc)
            print(f"{layout} reach {reach} ({rep.cell_reach}), {label}: pairs {rep.pairs_direct:.0f} / {nd}, "
                  f"images {rep.pairs_image:.0f} / {ni}")
            assert nd > 0 and ni > 0
            assert int(rep.pairs_direct) == nd
            assert int(rep.pairs_image) == ni
    finally:
        c.close()


def _rel(a, b, ref):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(ref ** 2)))


@pytest.mark.parametrize("layout", ["uniform", "clustered"])
@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("prec", [1, 2])
def test_real_and_fourier_parts_against_the_oracle_split(layout, family, prec):
    """The split of Sec. 4 checked part by part (Sec. 6 measures the error the
    same way: the real-space part is exact up to rounding, so the whole error
    is the Fourier part's).  The GPU's real-space part (pairs within r_c,
    their images and corrections, the stokeslet's self term) against the
    oracle's, summed with the same kernels S_R, T_R, W_R and G_R; its
    Fourier part (spreading, transforms, scaling, quadrature) against the
    oracle's whole sum minus its real-space part; and the two parts against
    the whole evaluation."""
    n, t = 700, 400
    tol = 1e-10 if prec == 1 else 1e-5
    y, s = workloads.make(family, n, workloads.SEED_BASE + 80, layout=layout)
    xs, _ = workloads.make(family, t, workloads.SEED_BASE + 81, layout=layout)
    xs[:20] = y[:20]  # targets on sources: the pair is left out (and the self term added)
    rc = (120 * 3.0 / (4.0 * np.pi * n)) ** (1.0 / 3.0) * (0.5 if layout == "clustered" else 1.0)
    xi = ehs.xi_for_cutoff(family, rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, prec)
        yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
        for label, x in (("targets = sources", y), ("separate targets", xs)):
            xd = yd if x is y else torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
            u = {}
            for part in (0, 1, 2):
                c.set_option(ehs.OPT_PARTS, part)
                u[part] = c.evaluate(family, yd, sd, xd, xi, rc, tol).cpu().numpy()
            c.set_option(ehs.OPT_PARTS, 0)
            ref = oracle.halfspace(family, y, s, x)
            ref_r = oracle.ewald_real(family, y, s, x, xi, rc)
            e_r = _rel(u[1], ref_r, ref_r)
            e_f = _rel(u[2], ref - ref_r, ref)
            e_w = _rel(u[0], ref, ref)
            e_s = _rel(u[1] + u[2], u[0], u[0])
            print(f"{family} {layout} prec {prec}, {label}: real {e_r:.2e}, Fourier {e_f:.2e}, whole {e_w:.2e}, "
                  f"parts vs whole {e_s:.2e}")
            assert e_r <= (1e-13 if prec == 1 else 1e-6)
            assert e_f <= tol
            assert e_w <= tol
            assert e_s <= (1e-14 if prec == 1 else 1e-7)
    finally:
        c.close()


# ---------------------------------------------------------------------------
# spreading and quadrature (steps 5 and 10 of Algorithm 1) against a plain
# CPU Gaussian gridding in the geometry of the report
# ---------------------------------------------------------------------------
def _window(rep, P, z):
    """Per axis, the P grid nodes nearest to z (P/2 on either side) and the
    signed offsets node - z; the window must lie inside the M~ x M~ x 2M~ grid."""
    o, h, Mt = np.array(rep.origin), rep.h, rep.Mt
    base = np.floor((z - o) / h).astype(np.int64) - P // 2 + 1
    dims = np.array([Mt, Mt, 2 * Mt])
    assert np.all(base >= 0) and np.all(base + P <= dims), "support outside the grid"
    idx = base[:, None] + np.arange(P)[None, :]
    return idx, o[:, None] + idx * h - z[:, None]


def _w1(rep, d):
    """1D factors of W(d) = (2 xi^2/(pi eta))^{3/2} exp(-2 xi^2 |d|^2/eta)
    and of its first and second derivatives with respect to the node."""
    a = 2.0 * rep.xi ** 2 / rep.eta
    w = np.exp(-a * d * d)
    return w, -2.0 * a * d * w, (4.0 * a * a * d * d - 2.0 * a) * w


def _sym(g, q):
    """sym(g q^T) as (xx, xy, xz, yy, yz, zz)."""
    return np.array([g[0] * q[0], 0.5 * (g[0] * q[1] + g[1] * q[0]), 0.5 * (g[0] * q[2] + g[2] * q[0]),
                     g[1] * q[1], 0.5 * (g[1] * q[2] + g[2] * q[1]), g[2] * q[2]])


def _cpu_spread(family, rep, y, s, n_spread, free):
    """The grids spread from the sources, their images y^I = (y1, y2, -y3)
    and the correction sources at the images (Sec. 3), each point's strengths
    times W on its P^3 window; with a density (report dgrid), the correction
    sources enter as one grid with derivatives of W."""
    Mt, P = rep.Mt, rep.Ps
    G = np.zeros((n_spread, 2 * Mt, Mt, Mt))
    pref = (2.0 * rep.xi ** 2 / (np.pi * rep.eta)) ** 1.5
    R = np.array([1.0, 1.0, -1.0])
    for m in range(len(y)):
        if family == "stokeslet":
            f = s[m]
            a_src, a_img = f, -f * R  # f at y, -f^I at y^I
            corr = [f[2], *(y[m, 2] * f * R)]  # C2 = f3, C3 = y3 f^I
        elif family == "stresslet":
            S = _sym(s[m, :3], s[m, 3:])
            SI = S * np.array([1, 1, -1, 1, -1, 1])  # R S R
            a_src, a_img = S, -SI
            corr = [S[0] + S[3] + S[5], *(y[m, 2] * SI)]  # C2 = g.q, C3 = y3 sym(g^I q^I)
        else:
            v = s[m]
            a_src, a_img = v, v * R
            corr = [-2.0 * v[1], 2.0 * v[0]]  # C2 = 2 (e3 x v) restricted to x1, x2
        for img in ((False,) if free else (False, True)):
            z = y[m] * (R if img else 1.0)
            idx, d = _window(rep, P, z)
            w = [_w1(rep, d[a]) for a in range(3)]
            sl = np.ix_(idx[2], idx[1], idx[0])
            W = pref * np.einsum("k,j,i->kji", w[2][0], w[1][0], w[0][0])
            ca = a_img if img else a_src
            for c in range(len(ca)):
                G[c][sl] += ca[c] * W
            if not img:
                continue
            nA = len(ca)
            if not rep.dgrid:
                for c in range(len(corr)):
                    G[nA + c][sl] += corr[c] * W
                continue
            def dW(ax, ay, az):  # derivative orders per axis
                return pref * np.einsum("k,j,i->kji", w[2][az], w[1][ay], w[0][ax])
            if family == "stokeslet":  # D = -2 C2 - 2 div C3
                D = -2.0 * (corr[0] * dW(0, 0, 0) + corr[1] * dW(1, 0, 0) + corr[2] * dW(0, 1, 0)
                            + corr[3] * dW(0, 0, 1))
            elif family == "stresslet":  # D = 4 d3 C2 - 4 grad grad : C3
                c3 = corr[1:]
                D = 4.0 * corr[0] * dW(0, 0, 1) - 4.0 * (
                    c3[0] * dW(2, 0, 0) + 2 * c3[1] * dW(1, 1, 0) + 2 * c3[2] * dW(1, 0, 1)
                    + c3[3] * dW(0, 2, 0) + 2 * c3[4] * dW(0, 1, 1) + c3[5] * dW(0, 0, 2))
            else:  # D = 2 div C2
                D = 2.0 * (corr[0] * dW(1, 0, 0) + corr[1] * dW(0, 1, 0))
            G[nA][sl] += D
    return G


def _cpu_quadrature(rep, G, x, free, fp64):
    """u(x) = h^3 sum over the Pg^3 window of W(node - x) times the velocity
    grids, less x3 times the gradient of phi: by derivative weights from the
    phi grid (FP64) or from the three grad phi grids (FP32)."""
    pref = (2.0 * rep.xi ** 2 / (np.pi * rep.eta)) ** 1.5
    h3 = rep.h ** 3
    u = np.zeros((len(x), 3))
    for t in range(len(x)):
        idx, d = _window(rep, rep.Pg, x[t])
        w = [_w1(rep, -d[a]) for a in range(3)]  # derivatives with respect to the target
        sl = np.ix_(idx[2], idx[1], idx[0])
        W = pref * np.einsum("k,j,i->kji", w[2][0], w[1][0], w[0][0])
        for a in range(3):
            u[t, a] = np.sum(W * G[a][sl])
        if free:
            continue
        if fp64:
            ph = G[3][sl]
            grads = [pref * np.einsum("k,j,i->kji", w[2][0], w[1][0], w[0][1]),
                     pref * np.einsum("k,j,i->kji", w[2][0], w[1][1], w[0][0]),
                     pref * np.einsum("k,j,i->kji", w[2][1], w[1][0], w[0][0])]
            for a in range(3):
                u[t, a] -= x[t, 2] * np.sum(grads[a] * ph)
        else:
            for a in range(3):
                u[t, a] -= x[t, 2] * np.sum(W * G[3 + a][sl])
    return h3 * u


@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("mode", ["fp64-grids", "fp64-density", "fp32", "free"])
@pytest.mark.parametrize("n_targets", [40, 3000])
def test_spreading_and_quadrature_against_plain_gridding(family, mode, n_targets):
    n = 60
    y, s = workloads.make(family, n, workloads.SEED_BASE + 90)
    x, _ = workloads.make(family, n_targets, workloads.SEED_BASE + 91)
    fp64 = mode != "fp32"
    free = mode == "free"
    tol = 1e-8 if fp64 else 1e-5
    rc = 0.3
    xi = ehs.xi_for_cutoff(family, rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1 if fp64 else 2)
        c.set_option(ehs.OPT_DGRID, 1 if mode == "fp64-density" else 0)
        yd, sd, xd = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (y, s, x))
        r = c.debug_grid_taps(family, yd, sd, xd, xi, rc, tol, free_space=free)
        rep = r["report"]
        assert rep.dgrid == (1 if mode == "fp64-density" else 0)
        G = r["spread"].cpu().numpy()
        ref = _cpu_spread(family, rep, y, s, r["n_spread"], free)
        e_s = np.max(np.abs(G - ref)) / np.max(np.abs(ref))
        g = np.random.default_rng(92)
        Q = g.standard_normal((r["n_quad"], 2 * rep.Mt, rep.Mt, rep.Mt))
        rq = c.debug_grid_taps(family, yd, sd, xd, xi, rc, tol, free_space=free, quad_in=torch.from_numpy(Q).to(DEV))
        uq = rq["u"].cpu().numpy()
        refq = _cpu_quadrature(rep, Q, x, free, fp64)
        e_q = np.max(np.abs(uq - refq)) / np.max(np.abs(refq))
        nodes = rep.Mt ** 3 * 2
        print(f"{family} {mode} T={n_targets}: Mt={rep.Mt} Ps={rep.Ps} Pg={rep.Pg} "
              f"node-owner quadrature={'yes' if (not free and rep.Pg >= 16 and n_targets < 3e-3 * nodes) else 'no'}"
              f" spread {e_s:.2e} quadrature {e_q:.2e}")
        bound = 1e-12 if fp64 else 2e-5
        assert e_s <= bound
        assert e_q <= bound
    finally:
        c.close()


@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("prec", [1, 2])
def test_quadrature_of_clustered_repeated_and_wall_targets(family, prec):
    """The grouped quadrature where targets crowd: 4000 targets clustered at
    the wall, 300 of them repeated (equal points in one group) and 50 on the
    wall itself (x3 = 0), against the plain CPU quadrature."""
    n = 60
    y, s = workloads.make(family, n, workloads.SEED_BASE + 93)
    x, _ = workloads.make(family, 4000, workloads.SEED_BASE + 94, layout="clustered")
    g = np.random.default_rng(95)
    x[g.choice(len(x), 50, replace=False), 2] = 0.0
    x[1::13][:300] = x[0::13][:300]
    tol = 1e-8 if prec == 1 else 1e-5
    rc = 0.3
    xi = ehs.xi_for_cutoff(family, rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, prec)
        yd, sd, xd = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (y, s, x))
        r = c.debug_grid_taps(family, yd, sd, xd, xi, rc, tol)
        rep = r["report"]
        Q = g.standard_normal((r["n_quad"], 2 * rep.Mt, rep.Mt, rep.Mt))
        rq = c.debug_grid_taps(family, yd, sd, xd, xi, rc, tol, quad_in=torch.from_numpy(Q).to(DEV))
        uq = rq["u"].cpu().numpy()
        refq = _cpu_quadrature(rep, Q, x, False, prec == 1)
        e_q = np.max(np.abs(uq - refq)) / np.max(np.abs(refq))
        print(f"{family} prec {prec}: Mt={rep.Mt} Pg={rep.Pg} quadrature {e_q:.2e}")
        assert e_q <= (1e-12 if prec == 1 else 2e-5)
        # repeated targets agree to rounding (in one group bit for bit; a group
        # boundary between them changes the order of the sums)
        d = np.max(np.abs(uq[1::13][:300] - uq[0::13][:300])) / np.max(np.abs(refq))
        assert d <= (1e-13 if prec == 1 else 1e-5)
    finally:
        c.close()


def test_stage_hooks_refuse_bad_arguments():
    """EHS_OPT_PARTS takes 0, 1 or 2; the grid taps refuse a buffer smaller
    than the plan's grids (after planning, nothing written past it) and
    contexts created with an arena."""
    import ctypes

    y, s = workloads.make("stokeslet", 200, workloads.SEED_BASE + 96)
    xi = ehs.xi_for_cutoff("stokeslet", 0.3, 5e-9)
    c = ehs.Context(0)
    try:
        with pytest.raises(ehs.EhsError) as e:
            c.set_option(ehs.OPT_PARTS, 3)
        assert e.value.code == ehs.EHS_EINVAL
        yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
        r = c.debug_grid_taps("stokeslet", yd, sd, yd, xi, 0.3, 1e-8)
        need = r["spread"].numel()
        small = torch.full((need - 1 + 16,), 7.0, dtype=torch.float64, device=DEV)
        out = torch.empty((200, 3), dtype=torch.float64, device=DEV)
        counts = (ctypes.c_int32 * 2)()
        rc = ehs.lib().ehs_debug_grid_taps(c._h, ehs.STOKESLET, 0, ctypes.c_void_p(yd.data_ptr()),
                                           ctypes.c_void_p(sd.data_ptr()), 200, ctypes.c_void_p(yd.data_ptr()), 200,
                                           xi, 0.3, 1e-8, ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(small.data_ptr()), need - 1, None, 0, counts, None, None)
        torch.cuda.synchronize()
        assert rc == ehs.EHS_EINVAL
        assert torch.all(small[need - 1:] == 7.0)  # nothing past the stated size
        assert counts[0] == r["n_spread"]
        # the context still evaluates, with the taps cleared
        u = c.evaluate("stokeslet", yd, sd, yd, xi, 0.3, 1e-8)
        torch.cuda.synchronize()
        assert oracle.rel_rms(oracle.halfspace("stokeslet", y, s, y), u.cpu().numpy()) <= 1e-8
    finally:
        c.close()
    a = ehs.Context(0, arena_bytes=1 << 30)
    try:
        yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
        with pytest.raises(ehs.EhsError) as e:
            a.debug_grid_taps("stokeslet", yd, sd, yd, xi, 0.3, 1e-8)
        assert e.value.code == ehs.EHS_EINVAL
    finally:
        a.close()


@pytest.mark.parametrize("n_targets", [1, 2, 3, 5, 7, 4001])
@pytest.mark.parametrize("mode", ["fp32", "free"])
def test_quadrature_partial_groups(mode, n_targets):
    """Target counts that leave the last group of four short (FP32 and free
    space take the grouped quadrature whatever the density)."""
    n = 60
    y, s = workloads.make("rotlet", n, workloads.SEED_BASE + 97)
    x, _ = workloads.make("rotlet", n_targets, workloads.SEED_BASE + 98, layout="clustered")
    fp64 = mode == "free"
    tol = 1e-8 if fp64 else 1e-5
    xi = ehs.xi_for_cutoff("rotlet", 0.3, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1 if fp64 else 2)
        yd, sd, xd = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (y, s, x))
        r = c.debug_grid_taps("rotlet", yd, sd, xd, xi, 0.3, tol, free_space=mode == "free")
        rep = r["report"]
        g = np.random.default_rng(99)
        Q = g.standard_normal((r["n_quad"], 2 * rep.Mt, rep.Mt, rep.Mt))
        rq = c.debug_grid_taps("rotlet", yd, sd, xd, xi, 0.3, tol, free_space=mode == "free",
                               quad_in=torch.from_numpy(Q).to(DEV))
        uq = rq["u"].cpu().numpy()
        refq = _cpu_quadrature(rep, Q, x, mode == "free", fp64)
        e_q = np.max(np.abs(uq - refq)) / np.max(np.abs(refq))
        print(f"{mode} T={n_targets}: quadrature {e_q:.2e}")
        assert uq.shape == (n_targets, 3)
        assert e_q <= (1e-12 if fp64 else 2e-5)
    finally:
        c.close()
