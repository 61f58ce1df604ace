"""Host-side checks of the library (no GPU needed).

* the C ABI loads and exports every entry point that include/ehs.h declares;
* the truncated Green's function transforms (paper Sec. 5.2) against 1D
  radial quadrature and their k -> 0 limits;
* parameter selection (plan) invariants and argument errors.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest
from scipy import integrate

import paper_1802_07844_amd as ehs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ehs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:ehs|ewald)_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ehs.lib()
    syms = _declared_symbols()
    assert "ewald_halfspace_stokeslet" in syms and "ehs_create" in syms
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in ehs.h but not exported"


def test_strerror_codes():
    for code in (0, -1, -2, -3, -4, -5):
        assert len(ehs.strerror(code)) > 4
    assert "unknown" in ehs.strerror(-99)


def _quad_H(k, R):
    # FT of 1/r restricted to r < R: (4 pi / k) int_0^R sin(k r) dr
    v, _ = integrate.quad(lambda r: math.sin(k * r), 0.0, R, limit=400)
    return 4 * math.pi / k * v


def _quad_B(k, R):
    # FT of (r - R) restricted to r < R: (4 pi / k) int_0^R r (r - R) sin(k r) dr
    v, _ = integrate.quad(lambda r: r * (r - R) * math.sin(k * r), 0.0, R, limit=400)
    return 4 * math.pi / k * v


@pytest.mark.parametrize("R", [0.7, 2.449, 5.0])
@pytest.mark.parametrize("k", [1e-3, 0.05, 0.3, 1.0, 3.7, 12.0, 41.0])
def test_truncated_kernels_match_radial_quadrature(R, k):
    for kind, q in ((0, _quad_H), (1, _quad_B)):
        ref = q(k, R)
        got = ehs.truncated_kernel_hat(kind, k, R)
        scale = 2 * math.pi * R * R if kind == 0 else math.pi * R**4 / 3
        assert abs(got - ref) <= 1e-10 * scale, (kind, k, R, got, ref)


@pytest.mark.parametrize("R", [0.5, 2.449])
def test_truncated_kernels_limits_at_zero(R):
    assert ehs.truncated_kernel_hat(0, 0.0, R) == pytest.approx(2 * math.pi * R * R, rel=1e-15)
    assert ehs.truncated_kernel_hat(1, 0.0, R) == pytest.approx(-math.pi * R**4 / 3, rel=1e-15)
    # continuity across the switch between series and closed form (R k = 0.5)
    for kind in (0, 1):
        a = ehs.truncated_kernel_hat(kind, (0.5 - 1e-13) / R, R)
        b = ehs.truncated_kernel_hat(kind, (0.5 + 1e-13) / R, R)
        assert abs(a - b) <= 1e-12 * abs(a)


def test_xi_for_cutoff_monotone():
    xa = ehs.xi_for_cutoff("stokeslet", 0.1, 1e-10)
    xb = ehs.xi_for_cutoff("stokeslet", 0.1, 1e-5)
    xc = ehs.xi_for_cutoff("stokeslet", 0.2, 1e-10)
    assert xa > xb > 0 and xa > xc > 0
    # xi r_c of about 4.8 for 1e-10 (exp(-(xi r_c)^2) ~ 1e-10)
    assert 4.0 < xa * 0.1 < 5.5
    assert ehs.xi_for_cutoff("rotlet", -1.0, 1e-10) < 0


def _plan(family="stokeslet", tol=1e-10, xi=12.0, rc=0.4, n=1000, prec=0, lo=(0, 0, 0), hi=(1, 1, 1)):
    return ehs.plan_query(family, n, n, lo, hi, 3.0 * n, xi, rc, tol, prec)


def _smooth7(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_plan_invariants(family, tol):
    r = _plan(family, tol)
    # Gaussian support from exp(-pi P c^2 / 2) <= tol / 40 (tol / 4 for the FP32 stokeslet and
    # rotlet at tol >= 1e-6), c = 0.95; two more for the stresslet's correction density
    base = 20 if tol == 1e-10 else 12 if family == "stresslet" else 10
    assert r.P == base + (2 if (family == "stresslet" and r.dgrid) else 0)
    assert r.Mt % 2 == 0 and _smooth7(r.Mt) and r.Mt >= r.M + max(r.P, r.Pg)
    assert 0.0 < r.eta < 1.0
    assert r.precision == (1 if tol < 1e-5 else 2)
    assert r.h == pytest.approx(r.L / r.M)
    assert r.Lt == pytest.approx(r.Mt * r.h)
    assert r.est_fourier <= (tol / 40 if family == "rotlet" else tol / 4)
    # the wall is a grid node: origin x3 = -M~ h
    assert r.origin[2] == pytest.approx(-r.Lt)
    assert r.nf >= (1 + math.sqrt(6)) * r.Mt and r.nf3 >= (2 + math.sqrt(6)) * r.Mt
    assert r.workspace_bytes > 0


def test_plan_errors():
    with pytest.raises(ehs.EhsError) as e:
        _plan(tol=1e-1)
    assert e.value.code == ehs.EHS_EINVAL
    with pytest.raises(ehs.EhsError) as e:
        _plan(xi=-1.0)
    assert e.value.code == ehs.EHS_EINVAL
    # a grid far beyond the supported size
    with pytest.raises(ehs.EhsError) as e:
        _plan(xi=4000.0, rc=0.001)
    assert e.value.code == ehs.EHS_ERANGE


def test_plan_box_covers_points_and_margin():
    r = _plan(lo=(0.25, -0.5, 0), hi=(0.9, 0.2, 0.8))
    L = max(0.65, 0.7, 0.8)
    assert r.L == pytest.approx(L, rel=1e-9)
    # in-plane origin half the wider (quadrature) support below the lowest point
    pe = max(r.P, r.Pg)
    assert r.Pg == r.P + (2 if r.precision == 1 else 0)
    assert r.origin[0] == pytest.approx(0.25 - pe * r.h / 2)
    assert r.origin[1] == pytest.approx(-0.5 - pe * r.h / 2)
    # the screening margin: (M~ - M) h >= sqrt(2 ln(1/tol)) / (sqrt2 xi)
    assert (r.Mt - r.M) * r.h >= math.sqrt(2 * math.log(1e10)) / (math.sqrt(2) * 12.0) - 1e-12


def test_create_without_device_fails_cleanly():
    """On a host without a GPU, context creation returns an error code."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = ehs.lib().ehs_create(ctypes.byref(h), 0, 0)
    assert rc != 0 and not h.value


@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("prec", [1, 2])
def test_plan_sweep_passes_extent_audit(family, prec):
    """Every plan over a sweep of sizes passes the library's buffer-extent audit."""
    tol = 1e-10 if prec == 1 else 1e-5
    for n, t in ((1, 1), (2, 5), (300, 300), (1000, 77), (100_000, 100_000), (1_000_000, 1_000_000)):
        for nb in (30, 300, 2000):
            rc = (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
            xi = ehs.xi_for_cutoff(family, rc, tol)
            try:
                r = ehs.plan_query(family, n, t, (0, 0, 0), (1, 1, 1), 3.0 * n, xi, rc, tol, prec)
            except ehs.EhsError as e:
                # only "grid too large" is acceptable, never an internal inconsistency
                assert e.code == ehs.EHS_ERANGE
                assert (math.pi / (1.0 / 2048)) < 7 * xi or nb == 30
                continue
            assert r.workspace_bytes > 0 and r.Mt >= r.M + r.P


def test_server_create_without_device_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = ehs.lib().ehs_server_create(ctypes.byref(h), 0, 1 << 30, 2)
    assert rc != 0 and not h.value
    assert "timeout" in ehs.strerror(ehs.EHS_ETIMEDOUT)


def test_fp32_estimate_and_auto_precision():
    """Auto precision takes FP32 at tol >= 1e-5 only while the FP32 rounding
    estimate stays within tol/2; a forced FP32 run beyond it is flagged."""
    lo, hi = (0, 0, 0), (1, 1, 1)
    small = ehs.plan_query("stokeslet", 10**5, 10**5, lo, hi, 3e5, 30.0, 0.12, 1e-5, 0)
    large = ehs.plan_query("stokeslet", 10**5, 10**5, lo, hi, 3e5, 118.0, 0.0415, 1e-5, 0)
    assert small.precision == 2 and small.est_fp32 <= 0.5e-5 and not (small.warnings & 4)
    assert large.precision == 1 and large.est_fp32 > 0.5e-5
    forced = ehs.plan_query("stokeslet", 10**5, 10**5, lo, hi, 3e5, 118.0, 0.0415, 1e-5, 2)
    assert forced.precision == 2 and (forced.warnings & 4)
    # the estimate grows with xi L
    e = [ehs.plan_query("stokeslet", 1000, 1000, lo, hi, 3e3, x, 3.5 / x, 1e-5, 2).est_fp32 for x in (10, 30, 90)]
    assert e[0] < e[1] < e[2]
    # the rotlet's rounding does not grow with xi: FP32 stays available
    rot = ehs.plan_query("rotlet", 10**5, 10**5, lo, hi, 3e5, 118.0, 0.0415, 1e-5, 0)
    assert rot.precision == 2


@pytest.mark.parametrize("dgrid", [0, 1])
def test_record_region_holds_the_spreading_support(dgrid):
    """The workspace's record region is sized with the spreading support the
    kernels use (P + 2 when the correction
    density is spread with derivative weights): the audit passes, and the
    reported workspace grows with the record stride; the stresslet's density
    (second derivatives: P + 6) comes with two more support nodes in P."""
    n = 100_000
    for fam in ("stokeslet", "stresslet", "rotlet"):
        rc = (30 * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
        xi = ehs.xi_for_cutoff(fam, rc, 0.5e-10)
        r = ehs.plan_query(fam, n, n, (0, 0, 0), (1, 1, 1), 3.0 * n, xi, rc, 1e-10, 1)
        extra = 6 if fam == "stresslet" else 2
        assert r.Ps == (r.P + extra if r.dgrid else r.P)
        assert r.P == (22 if (fam == "stresslet" and r.dgrid) else 20)
        assert r.Pg == r.P + 2 and r.Mt >= r.M + max(r.Ps, r.Pg)
        stride = 2 + 3 * r.Ps + 3 + {"stokeslet": 7, "stresslet": 13, "rotlet": 5}[fam]
        assert r.workspace_bytes >= 2 * n * stride * 8


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("z0", [0.0, 0.3, 0.9])
def test_inverse_transforms_cover_the_lowest_target(prec, z0):
    """The inverse transforms produce x3 nodes from x3_first up; the Gaussian
    support of the lowest target (base floor((z - o3) / h) - Pg/2 + 1) must
    start at or above it, and the image half of the box below the wall is
    skipped."""
    r = _plan(lo=(0.0, 0.0, z0), hi=(1.0, 1.0, 1.0), prec=prec)
    first = math.floor((z0 - r.origin[2]) / r.h) - r.Pg // 2 + 1
    assert 0 <= r.x3_first <= first
    assert r.x3_first % 16 == 0
    assert r.x3_first >= first - 17  # one node of margin, rounded down to 16
    assert r.origin[2] == pytest.approx(-r.Lt)
    if z0 == 0.0:
        assert r.x3_first >= r.Mt - r.Pg // 2 - 17


@pytest.mark.parametrize("dgrid_family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("z0", [1e-4, 0.2, 0.6])
def test_correction_grids_end_above_the_highest_image_support(dgrid_family, z0):
    """The correction sources sit at the images, x3 = -y3 <= -z0: every node
    of their Gaussian support (top node floor((-z0 - o3) / h) + Ps/2) lies
    below x3_corr_end, which the forward transforms use as the end of those
    grids."""
    r = _plan(family=dgrid_family, lo=(0.0, 0.0, z0), hi=(1.0, 1.0, 1.0), prec=1)
    top = math.floor((-z0 - r.origin[2]) / r.h) + r.Ps // 2
    assert top < r.x3_corr_end <= 2 * r.Mt
    assert r.x3_corr_end <= top + 2 + 16
    assert r.x3_corr_end <= r.Mt + r.Ps // 2 + 18  # never above the wall's support


@pytest.mark.parametrize("n,nb", [(100_000, 30), (1_000_000, 2000), (4_000_000, 300)])
def test_real_space_cells_cover_the_cutoff(n, nb):
    """Cells have side >= r_c (3^3 walk) or, where cells of side r_c would
    hold 256 targets or more on average, side >= r_c / 2 (5^3 walk): either
    way the walked cells hold every source within r_c."""
    rc = (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    r = _plan(n=n, rc=rc, xi=ehs.xi_for_cutoff("stokeslet", rc, 0.5e-10), prec=1)
    L = [1.0, 1.0, 1.0]
    dense = n >= 256 * np.prod([max(1.0, math.floor(x / rc)) for x in L])
    reach = 2 if dense else 1
    for a in range(3):
        side = L[a] / r.ncell[a]
        assert side * reach >= rc * (1 - 1e-12)
        assert r.ncell[a] <= 256
    if dense:
        assert r.ncell[0] >= 2 * math.floor(1.0 / rc) - 1 or r.ncell[0] == 256


@pytest.mark.parametrize("family", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_cutoff_for_estimate_inverts_the_real_space_estimate(family, tol):
    """The tuner's cutoff at a given xi: the estimate there equals the target
    (checked through the planner's own estimate), and it inverts
    xi_for_cutoff; along xi the product xi r_c moves only logarithmically, as
    the tuning procedure of the results section assumes."""
    L = 1.0
    for rc in (0.03, 0.1, 0.3):
        xi = ehs.xi_for_cutoff(family, rc, tol, L)
        got = ehs.cutoff_for_estimate(family, xi, tol / 2, L)
        assert got == pytest.approx(rc, rel=1e-9)
        if rc == 0.3:  # a grid the planner admits at every tolerance
            rep = _plan(family, tol=tol, xi=xi, rc=got, n=2000, hi=(L, L, L))
            assert rep.est_real == pytest.approx(tol / 2, rel=1e-6)
    xi0 = ehs.xi_for_cutoff(family, 0.05, tol, L)
    p0 = xi0 * ehs.cutoff_for_estimate(family, xi0, tol / 2, L)
    prev = None
    for f in (0.5, 0.7071, 1.0, 1.4142, 2.0):
        rc = ehs.cutoff_for_estimate(family, f * xi0, tol / 2, L)
        assert rc > 0
        if prev is not None:
            assert rc < prev  # larger xi, smaller cutoff
        prev = rc
        assert f * xi0 * rc == pytest.approx(p0, rel=0.08)


def test_cutoff_for_estimate_bad_arguments():
    assert ehs.cutoff_for_estimate("stokeslet", -1.0, 1e-10) < 0
    assert ehs.cutoff_for_estimate("stokeslet", 10.0, 0.0) < 0
    assert ehs.cutoff_for_estimate(7, 10.0, 1e-10) < 0
    # an estimate above its value at xi r_c = 1 is out of range
    assert ehs.cutoff_for_estimate("stokeslet", 10.0, 10.0) < 0


def test_tune_rejects_bad_arguments_without_a_device():
    """Argument checks of ehs_tune come before any device work."""
    L = ehs.lib()
    best = (ctypes.c_double * 3)()
    assert L.ehs_tune(None, 0, None, None, 10, None, 10, 10.0, 0.3, 1e-10, 4, None, best, None, None, None,
                      None) == ehs.EHS_EINVAL


def _erfc_coefficients():
    import re

    text = open(os.path.join(ROOT, "paper_1802_07844_amd", "csrc", "erfc_poly.h")).read()
    out = {}
    for name in ("ERFC_C64", "ERFC_C32"):
        body = text.split(name + "[] = {", 1)[1].split("};", 1)[0]
        out[name] = [float(v.rstrip("f")) for v in re.findall(r"[-+0-9.eE]+f?", body)]
    return out


@pytest.mark.parametrize("name,dtype,bound", [("ERFC_C64", np.float64, 2e-15), ("ERFC_C32", np.float32, 6e-7)])
def test_erfc_polynomial_of_the_real_space_sum(name, dtype, bound):
    """The real-space kernels form erfc(x) = exp(-x^2) q(1 / (1 + x/2)) with
    the coefficients of erfc_poly.h: absolute error against a 30-digit erfc
    over every argument a cutoff can produce (0 <= x <= 6.5), evaluated in
    the kernels' precision with the same Horner order."""
    import mpmath as mp

    mp.mp.dps = 30
    c = [dtype(v) for v in _erfc_coefficients()[name]]
    assert len(c) == (15 if dtype == np.float64 else 8)
    g = np.random.default_rng(5)
    x = np.concatenate([np.linspace(0.0, 6.5, 1500), g.random(1500) * 6.5, [0.0, 1e-12, 6.5]]).astype(dtype)
    t = dtype(1) / (dtype(1) + dtype(0.5) * x)
    q = np.full_like(x, c[-1])
    for v in c[-2::-1]:
        q = q * t + v
    got = (np.exp(-x * x) * q).astype(np.float64)
    ref = np.array([float(mp.erfc(mp.mpf(float(v)))) for v in x])
    err = np.max(np.abs(got - ref))
    print(f"{name}: max |erfc error| = {err:.2e}")
    assert err <= bound


def test_stresslet_density_chosen_by_cost():
    """Auto mode takes the stresslet's correction density where the grid is
    large for the number of points (the saved transforms outweigh the wider
    support: measured 0.61-0.87 of the time from 130 grid nodes per point
    up) and the separate grids where the points dominate (1.07-1.37 below)."""
    def plan(n, nb, tol):
        rc = (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
        xi = ehs.xi_for_cutoff("stresslet", rc, tol / 2)
        return ehs.plan_query("stresslet", n, n, (0, 0, 0), (1, 1, 1), 1.0 * n, xi, rc, tol, 1)

    assert plan(100_000, 30, 1e-10).dgrid == 1
    assert plan(1_000_000, 600, 1e-10).dgrid == 1
    assert plan(1_000_000, 2000, 1e-10).dgrid == 0
    assert plan(1_000_000, 2000, 1e-5).dgrid == 0
    r = plan(1_000_000, 300, 1e-5)
    assert r.dgrid == 1 and r.P == 14 and r.Ps == 20


def test_plans_over_the_whole_tolerance_range():
    """Every family has an FP64 plan down to tol 1e-14, the bottom of the
    documented range.  Auto mode takes the correction density only from tol
    1e-12 up (its rounding floor is about 1e-13) and where its support fits:
    the stresslet's needs P + 8 spreading nodes, at most 30."""
    n = 400
    for fam in ("stokeslet", "stresslet", "rotlet"):
        for tol in (1e-12, 1e-13, 1e-14):
            rc = (120 * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
            xi = ehs.xi_for_cutoff(fam, rc, tol / 2)
            p = ehs.plan_query(fam, n, n, (0, 0, 0), (1, 1, 1), 1.0 * n, xi, rc, tol, 1)
            assert p.P <= 30 and p.Pg <= 30 and p.Ps <= 30
            if tol < 1e-12 or (fam == "stresslet" and p.P + 8 > 30):
                assert p.dgrid == 0


def _pair_exp_steps():
    """The constants of the FP64 real-space exponential, read from the source."""
    text = open(os.path.join(ROOT, "paper_1802_07844_amd", "csrc", "realspace.hip")).read()
    body = text.split("static __device__ __forceinline__ double exp(double y)", 1)[1].split("\n    }\n", 1)[0]
    log2e = float(re.search(r"rint\(y \* ([0-9.eE+-]+)\)", body).group(1))
    ln2 = [float(v) for v in re.findall(r"fma\(-k, ([0-9.eE+-]+),", body)]
    first = re.search(r"double p = ([0-9.]+) / ([0-9.]+);", body)
    coef = [float(first.group(1)) / float(first.group(2))]
    for num in re.findall(r"p = fma_sc\(p, f, ([^)]+?)\);", body):
        parts = num.split("/")
        coef.append(float(parts[0]) / float(parts[1]) if len(parts) == 2 else float(parts[0]))
    return log2e, ln2, coef


def _fma(a, b, c):
    # a fused multiply-add: the product and sum in 64-bit-mantissa
    # arithmetic, rounded once to double
    return (np.longdouble(a) * np.longdouble(b) + np.longdouble(c)).astype(np.float64)


def test_pair_arithmetic_of_the_real_space_sum():
    """The FP64 real-space kernels take 1/sqrt(x) and 1/x from the hardware
    estimates and one third-order Newton step, and e^y from a reduction by
    ln 2 and a Taylor series to f^12.  The same steps on the host, from
    estimates perturbed by 2^-21 (four times the estimates' stated error)
    and on every argument a pair can produce: within 4 ulp of the exact
    values, so the kernels' pair terms are as accurate as with the library
    functions."""
    import mpmath as mp

    mp.mp.dps = 40
    g = np.random.default_rng(11)
    eps = np.finfo(np.float64).eps
    # 1/sqrt(x) over the squared distances of pairs (positions in a unit box)
    x = np.concatenate([10.0 ** g.uniform(-12, 0.5, 4000), [1e-12, 1.0, 3.0]])
    for d in (2.0 ** -21, -(2.0 ** -21)):
        y = (1.0 / np.sqrt(x)) * (1.0 + d)
        e = _fma(-x * y, y, 1.0)
        r = _fma(y * e, _fma(e, 0.375, 0.5), y)
        ref = np.array([float(1 / mp.sqrt(mp.mpf(float(v)))) for v in x])
        assert np.max(np.abs(r - ref) / ref) <= 4 * eps
    # 1/x for x = 1 + xi r / 2 in [1, 8]
    x = np.concatenate([g.uniform(1.0, 8.0, 4000), [1.0, 8.0]])
    for d in (2.0 ** -21, -(2.0 ** -21)):
        y = (1.0 / x) * (1.0 + d)
        e = _fma(-x, y, 1.0)
        r = _fma(y * e, 1.0 + e, y)
        assert np.max(np.abs(r - 1.0 / x) * x) <= 4 * eps
    # e^y for y = -(xi r)^2 down to -(6.5)^2 and beyond
    log2e, ln2, coef = _pair_exp_steps()
    assert len(ln2) == 2 and len(coef) == 13
    assert abs(ln2[0] + ln2[1] - math.log(2.0)) < 1e-25 + 1e-16 * math.log(2.0)
    y = np.concatenate([-g.uniform(0.0, 60.0, 4000), [0.0, -1e-300, -42.25, -60.0]])
    k = np.rint(y * log2e)
    f = _fma(-k, ln2[0], y)
    f = _fma(-k, ln2[1], f)
    p = np.full_like(f, coef[0])
    for c in coef[1:]:
        p = _fma(p, f, c)
    r = np.ldexp(p, k.astype(int))
    ref = np.array([float(mp.exp(mp.mpf(float(v)))) for v in y])
    assert np.max(np.abs(r - ref) / ref) <= 4 * eps


def test_header_constants_match_the_binding():
    """Every option, error code, stage index and size constant that
    include/ehs.h defines has the same value in the Python binding."""
    text = open(os.path.join(ROOT, "include", "ehs.h")).read()
    defs = {}
    for name, val in re.findall(r"#define (EHS_\w+)\s+(\(\(size_t\)\d+ << \d+\)|\(?[-0-9]+\)?)", text):
        if "<<" in val:
            a, b = re.findall(r"(\d+) << (\d+)", val)[0]
            defs[name] = int(a) << int(b)
        else:
            defs[name] = int(val.strip("()"))
    opts = {k: v for k, v in defs.items() if k.startswith("EHS_OPT_")}
    assert len(opts) >= 12
    for k, v in opts.items():
        assert getattr(ehs, k[4:]) == v, k
    for k in ("EHS_OK", "EHS_EINVAL", "EHS_EDOMAIN", "EHS_ERANGE", "EHS_ENOMEM", "EHS_EHIP", "EHS_ETIMEDOUT",
              "EHS_ETOOBIG"):
        assert getattr(ehs, k) == defs[k], k
    stages = {k[7:].lower(): v for k, v in defs.items() if k.startswith("EHS_ST_")}
    assert defs["EHS_NSTAGES"] == len(ehs.STAGES)
    names = {"bbox": "bbox", "precomp": "precompute", "bin": "binning", "real": "realspace", "spread": "spread",
             "fwdx": "fwd_x", "fwdy": "fwd_y", "zscale": "z_scale", "invy": "inv_y", "invx": "inv_x",
             "gather": "gather", "total": "total"}
    for k, v in stages.items():
        assert ehs.STAGES[v] == names[k], k
    assert ehs.ARENA_MIN_BYTES == defs["EHS_ARENA_MIN_BYTES"]
    assert ehs.NOALLOC_SCRATCH_BYTES == defs["EHS_NOALLOC_SCRATCH_BYTES"]
