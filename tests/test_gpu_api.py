"""GPU tests of the context's memory behaviour and failure paths.

* A context created with an arena (ehs_create with arena_bytes > 0) takes
  every evaluation's tables, octants and workspace from that one region: its
  results equal those of a growing context, and the calls allocate nothing.
* A failed truncated-kernel precompute (forced from the host with the
  EHS_OPT_FAIL_PRECOMPUTE hook, before anything is launched) leaves no cache
  entry behind, in a context and in a server: the next call succeeds.
* The runtime-optimal search keeps only the fastest candidate's octants.
* The correction-density option (EHS_OPT_DGRID) in both settings against the
  oracle, for the stresslet with its larger support.
* The forcing options (M, P, M~, the quadrature's extra support, the slab
  groups of the transform pipeline): reflected in the report, within tol of
  the oracle, and refused out of range.
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


def _rc(nb, n):
    return (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)


def _problem(fam, n, seed, nb=300, tol=1e-10):
    y, s = workloads.make(fam, n, seed)
    rc = _rc(nb, n)
    xi = ehs.xi_for_cutoff(fam, rc, tol / 2)
    return y, s, torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV), xi, rc


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("prec", [1, 2])
def test_arena_context_matches_growing_context(prec):
    """Same plans, same arithmetic: bitwise-equal results from the arena
    context and the growing one, over calls whose grid size changes; the arena
    context's calls leave device memory unchanged."""
    tol = 1e-10 if prec == 1 else 1e-5
    grow = ehs.Context(0)
    arena = ehs.Context(0, arena_bytes=3 << 30)
    try:
        for c in (grow, arena):
            c.set_option(ehs.OPT_PRECISION, prec)
        cases = [("stokeslet", 1000, 51), ("rotlet", 400, 52), ("stresslet", 700, 53), ("stokeslet", 300, 54)]
        data = [_problem(f, n, sd, tol=tol) for f, n, sd in cases]
        outs = [torch.empty((yd.shape[0], 3), dtype=torch.float64, device=DEV) for _, _, yd, _, _, _ in data]
        ref = []
        for (fam, n, _), (y, s, yd, sd, xi, rc) in zip(cases, data):
            ref.append(grow.evaluate(fam, yd, sd, yd, xi, rc, tol).cpu().numpy())
        before = _free()
        for (fam, n, _), (y, s, yd, sd, xi, rc), o, r in zip(cases, data, outs, ref):
            u, rep = arena.evaluate(fam, yd, sd, yd, xi, rc, tol, out=o, report=True)
            torch.cuda.synchronize()
            got = u.cpu().numpy()
            print(f"arena {fam} N={n} prec={rep.precision} Mt={rep.Mt} zslab={rep.zslab} "
                  f"max|diff|={np.max(np.abs(got - r)):.2e}")
            assert rep.precision == prec
            np.testing.assert_array_equal(got, r)
        after = _free()
        print(f"device memory change over the arena calls: {(before - after) / 2**20:.1f} MiB")
        assert before - after < 32 * 2**20
        # and against the oracle, for the first case
        y, s = data[0][0], data[0][1]
        assert oracle.rel_rms(oracle.halfspace("stokeslet", y, s, y), ref[0]) <= tol
    finally:
        grow.close()
        arena.close()


def test_arena_context_too_small():
    arena = ehs.Context(0, arena_bytes=ehs.ARENA_MIN_BYTES)
    try:
        y, s, yd, sd, xi, rc = _problem("stokeslet", 1000, 55)
        with pytest.raises(ehs.EhsError) as e:
            arena.evaluate("stokeslet", yd, sd, yd, xi, rc, 1e-10)
        assert e.value.code == ehs.EHS_ENOMEM
    finally:
        arena.close()
    with pytest.raises(ehs.EhsError) as e:
        ehs.Context(0, arena_bytes=1 << 20)
    assert e.value.code == ehs.EHS_EINVAL


@pytest.mark.parametrize("arena_bytes", [0, 2 << 30])
def test_failed_precompute_leaves_no_cache_entry(arena_bytes):
    c = ehs.Context(0, arena_bytes=arena_bytes)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        y, s, yd, sd, xi, rc = _problem("stokeslet", 800, 56)
        c.set_option(ehs.OPT_FAIL_PRECOMPUTE, 1)
        with pytest.raises(ehs.EhsError) as e:
            c.evaluate("stokeslet", yd, sd, yd, xi, rc, 1e-10)
        assert e.value.code == ehs.EHS_EHIP
        if arena_bytes == 0:
            assert c.memory()["cache_entries"] == 0
        u, rep = c.evaluate("stokeslet", yd, sd, yd, xi, rc, 1e-10, report=True)
        torch.cuda.synchronize()
        assert rep.warnings & 2  # produced again in this call
        err = oracle.rel_rms(oracle.halfspace("stokeslet", y, s, y), u.cpu().numpy())
        print(f"after a failed precompute (arena {arena_bytes}): rel-RMS {err:.2e}")
        assert err <= 1e-10
    finally:
        c.close()


def test_server_recovers_after_failed_production():
    """One octant production fails: that request fails, the failed octant leaves
    the cache, and the next request with the same grid size succeeds."""
    y, s, yd, sd, xi, rc = _problem("rotlet", 900, 57)
    with ehs.Server(0, arena_bytes=2 << 30, nslots=1) as srv:
        srv.set_option(ehs.OPT_FAIL_PRECOMPUTE, 1)
        t = srv.submit("rotlet", yd, sd, yd, xi, rc, 1e-10, precision=1)
        with pytest.raises(ehs.EhsError) as e:
            srv.wait(t)
        assert e.value.code == ehs.EHS_EHIP
        st = srv.stats()
        assert st["failed"] == 1 and st["cache_entries"] == 0 and st["arena_used"] == 0
        t = srv.submit("rotlet", yd, sd, yd, xi, rc, 1e-10, precision=1)
        u, status = srv.wait(t)
        assert status["code"] == ehs.EHS_OK
        err = oracle.rel_rms(oracle.halfspace("rotlet", y, s, y), u.cpu().numpy())
        print(f"server after a failed production: rel-RMS {err:.2e}, stats {srv.stats()}")
        assert err <= 1e-10
        assert srv.stats()["cache_entries"] == 1


def test_tune_keeps_only_the_fastest_candidates_octants():
    n = 20_000
    y, f, yd, fd, xi, rc = _problem("stokeslet", n, 58, nb=60)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        res = c.tune("stokeslet", yd, fd, yd, xi, rc, 1e-10, max_evals=12)
        m = c.memory()
        print(f"tune: {len(res['trace'])} candidates, best xi={res['xi']:.2f} r_c={res['r_c']:.4f}; memory {m}")
        assert len(res["trace"]) >= 3
        assert m["cache_entries"] == 1
        assert m["cache_bytes"] <= 2 * 8 * (res["report"].Mt + 1) ** 2 * (2 * res["report"].Mt + 1)
    finally:
        c.close()


@pytest.mark.parametrize("fam", ["stokeslet", "rotlet"])
@pytest.mark.parametrize("dgrid", [0, 1])
def test_correction_density_option(fam, dgrid):
    n = 3000
    y, s, yd, sd, xi, rc = _problem(fam, n, 59 + dgrid)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        c.set_option(ehs.OPT_DGRID, dgrid)
        u, rep = c.evaluate(fam, yd, sd, yd, xi, rc, 1e-10, report=True)
        torch.cuda.synchronize()
        err = oracle.rel_rms(oracle.halfspace(fam, y, s, y), u.cpu().numpy())
        print(f"{fam} dgrid={dgrid}: plan dgrid={rep.dgrid} Ps={rep.Ps} rel-RMS {err:.2e}")
        assert rep.dgrid == dgrid
        assert err <= 1e-10
    finally:
        c.close()


@pytest.mark.parametrize("n,nb,tol", [(100_000, 30, 1e-10), (100_000, 300, 1e-10), (1_000_000, 300, 1e-5)])
def test_stresslet_correction_density(n, nb, tol):
    """The stresslet's correction density (second-derivative weights), on
    request, with the two extra support nodes it needs, in FP64 against the
    oracle on a sample; the separate-grid plan of the same points beside it."""
    y, s = workloads.make("stresslet", n, 61)
    rc = _rc(nb, n)
    xi = ehs.xi_for_cutoff("stresslet", rc, tol / 2)
    yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
    idx = np.sort(workloads.rng(67).choice(n, 256, replace=False))
    ref = oracle.halfspace("stresslet", y, s, y[idx])
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        c.set_option(ehs.OPT_TIMING, 1)
        out = {}
        for dg in (0, 1):
            c.set_option(ehs.OPT_DGRID, dg)
            u, rep = c.evaluate("stresslet", yd, sd, yd, xi, rc, tol, report=True)
            u, rep = c.evaluate("stresslet", yd, sd, yd, xi, rc, tol, report=True)  # timed without the precompute
            torch.cuda.synchronize()
            err = oracle.rel_rms(ref, u.cpu().numpy()[idx])
            out[dg] = (err, rep)
            print(f"stresslet N={n} ~{nb} neighbours tol {tol:g} dgrid={rep.dgrid}: P={rep.P} Ps={rep.Ps} "
                  f"Mt={rep.Mt} rel-RMS {err:.2e}, {rep.ms_stage[ehs.STAGES.index('total')]:.1f} ms")
            assert rep.dgrid == dg
            assert err <= tol
        assert out[1][1].P == out[0][1].P + 2
    finally:
        c.close()


@pytest.mark.parametrize("reach", [0, 1, 2, 3])
def test_cell_reach(reach):
    """Real-space cells of side r_c / reach (0: chosen from the targets'
    height histogram) on a set clustered at the wall: the same sum."""
    n = 20_000
    y, f = workloads.clustered_stokeslet(n, 62)
    rc, tol = 0.08, 1e-10
    xi = ehs.xi_for_cutoff("stokeslet", rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        c.set_option(ehs.OPT_TIMING, 1)
        c.set_option(ehs.OPT_CELL_REACH, reach)
        yd, fd = torch.from_numpy(y).to(DEV), torch.from_numpy(f).to(DEV)
        u, rep = c.evaluate("stokeslet", yd, fd, yd, xi, rc, tol, report=True)
        torch.cuda.synchronize()
        err = oracle.rel_rms(oracle.halfspace("stokeslet", y, f, y), u.cpu().numpy())
        print(f"reach {reach}: cell_reach={rep.cell_reach} occupancy={rep.occupancy:.1f} "
              f"pairs {rep.pairs_direct:.0f} + {rep.pairs_image:.0f} images, rel-RMS {err:.2e}")
        if reach:
            assert rep.cell_reach == reach
        assert rep.pairs_direct > 0 and rep.pairs_image > 0
        assert err <= tol
    finally:
        c.close()


@pytest.mark.parametrize("fam", ["stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("tol", [1e-5, 1e-7])
def test_fp64_at_loose_tolerances(fam, tol):
    """FP64 at tolerances looser than 1e-10 (auto precision picks FP64 at
    tol >= 1e-5 where the FP32 rounding estimate is too large): the error
    against the oracle stays within tol.  The FP64 path forms the correction
    gradient by quadrature with grad W, whose grid aliasing error is larger
    than W's, so its Gaussian support comes from the tighter budget."""
    for nb in (30, 300):
        n = 20_000
        y, s = workloads.make(fam, n, 63)
        rc = _rc(nb, n)
        xi = ehs.xi_for_cutoff(fam, rc, tol / 2)
        c = ehs.Context(0)
        try:
            c.set_option(ehs.OPT_PRECISION, 1)
            yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
            u, rep = c.evaluate(fam, yd, sd, yd, xi, rc, tol, report=True)
            torch.cuda.synchronize()
            idx = np.sort(workloads.rng(64).choice(n, 1024, replace=False))
            err = oracle.rel_rms(oracle.halfspace(fam, y, s, y[idx]), u.cpu().numpy()[idx])
            print(f"{fam} FP64 tol {tol:g} ~{nb} neighbours: P={rep.P} Pg={rep.Pg} Mt={rep.Mt} rel-RMS {err:.2e}")
            assert err <= tol
        finally:
            c.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_repeated_evaluations_are_bitwise_equal(prec):
    """The real-space sum adds its pair contributions to per-target LDS
    accumulators; the order of those adds is fixed by the wavefront's
    instructions, so two evaluations of the same input agree bit for bit
    (dense clustered set: hundreds of pairs per target)."""
    n = 60_000
    y, f = workloads.clustered_stokeslet(n, 65)
    tol = 1e-10 if prec == 1 else 1e-5
    rc = 0.06
    xi = ehs.xi_for_cutoff("stokeslet", rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, prec)
        yd, fd = torch.from_numpy(y).to(DEV), torch.from_numpy(f).to(DEV)
        u1 = c.evaluate("stokeslet", yd, fd, yd, xi, rc, tol).cpu().numpy()
        u2 = c.evaluate("stokeslet", yd, fd, yd, xi, rc, tol).cpu().numpy()
        np.testing.assert_array_equal(u1, u2)
        idx = np.sort(workloads.rng(66).choice(n, 256, replace=False))
        err = oracle.rel_rms(oracle.halfspace("stokeslet", y, f, y[idx]), u1[idx])
        print(f"clustered N={n} prec={prec}: rel-RMS {err:.2e}, repeat bitwise equal")
        assert err <= tol
    finally:
        c.close()


@pytest.mark.parametrize("fam,prec,free", [("stokeslet", 1, False), ("stresslet", 1, False), ("rotlet", 2, False),
                                           ("stokeslet", 1, True)])
def test_overlapped_real_space_sum_is_bitwise_the_same(fam, prec, free):
    """EHS_OPT_OVERLAP runs the real-space sum on the context's side stream
    beside the grid stages; the arithmetic is the same, so the results equal
    those of the serial order bit for bit, on the caller's default stream and
    on a stream of its own, and the timed report gives the sum its own time."""
    n = 30_000
    y, s = workloads.make(fam, n, workloads.SEED_BASE + 80, layout="clustered")
    tol = 1e-10 if prec == 1 else 1e-5
    rc = 0.06
    xi = ehs.xi_for_cutoff(fam, rc, tol / 2)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, prec)
        c.set_option(ehs.OPT_TIMING, 1)
        yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
        out = {}
        for ov in (0, 1):
            c.set_option(ehs.OPT_OVERLAP, ov)
            u, rep = c.evaluate(fam, yd, sd, yd, xi, rc, tol, report=True, free_space=free)
            torch.cuda.synchronize()
            out[ov] = (u.cpu().numpy(), rep.as_dict()["ms_stage"])
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            u3 = c.evaluate(fam, yd, sd, yd, xi, rc, tol, free_space=free, stream=st)
        st.synchronize()
        print(f"{fam} prec={prec} free={free}: real space {out[0][1]['realspace']:.2f} ms serial, "
              f"{out[1][1]['realspace']:.2f} ms overlapped; total {out[0][1]['total']:.2f} -> {out[1][1]['total']:.2f} ms")
        np.testing.assert_array_equal(out[0][0], out[1][0])
        np.testing.assert_array_equal(out[0][0], u3.cpu().numpy())
        assert out[1][1]["realspace"] > 0 and out[1][1]["total"] > 0
        with pytest.raises(ehs.EhsError):
            c.set_option(ehs.OPT_OVERLAP, 2)
    finally:
        c.close()


def _next_smooth_even(n):
    def smooth(m):
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        return m == 1

    while n % 2 or not smooth(n):
        n += 1
    return n


@pytest.mark.parametrize("family,prec", [("stokeslet", 1), ("stresslet", 1), ("rotlet", 2)])
def test_forced_plan_parameters(family, prec):
    """Forcing M, P, M~ or the quadrature's extra support shows in the report
    and, since each only adds grid or support, keeps the result within tol of
    the oracle; the slab grouping of the y / x3 transform pipeline (one k1
    slab at a time, or the whole grid at once) changes no bit of it."""
    tol = 1e-10 if prec == 1 else 1e-5
    y, s, yd, sd, xi, rc = _problem(family, 600, 77, nb=200, tol=tol)
    ref = oracle.halfspace(family, y, s, y)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, prec)
        u0, r0 = c.evaluate(family, yd, sd, yd, xi, rc, tol, report=True)
        u0 = u0.cpu().numpy()
        assert oracle.rel_rms(ref, u0) <= tol

        def run(opt, val, reset):
            c.set_option(opt, val)
            try:
                u, r = c.evaluate(family, yd, sd, yd, xi, rc, tol, report=True)
                return u.cpu().numpy(), r
            finally:
                c.set_option(opt, reset)

        for zg in (1, r0.Mt + 1):
            u, r = run(ehs.OPT_ZSLAB, zg, 0)
            assert r.zslab == zg
            assert np.array_equal(u, u0), f"slab groups of {zg}"
        dp = 4 if max(r0.P, r0.Pg) + 4 <= 30 else 2
        mt = _next_smooth_even(r0.Mt + 20)
        checks = [
            (ehs.OPT_FORCE_P, r0.P + dp, 0, lambda r: r.P == r0.P + dp),
            (ehs.OPT_FORCE_M, r0.M + 10, 0, lambda r: r.M == r0.M + 10),
            (ehs.OPT_FORCE_MT, mt, 0, lambda r: r.Mt == mt and r.M == r0.M),
            (ehs.OPT_GATHER_EXTRA, r0.Pg - r0.P + 2, -1, lambda r: r.Pg == r0.Pg + 2),
        ]
        for opt, val, reset, ok in checks:
            u, r = run(opt, val, reset)
            err = oracle.rel_rms(ref, u)
            print(f"{family} prec {prec}: option {opt} = {val}: M {r.M} P {r.P} Pg {r.Pg} Mt {r.Mt} rel-RMS {err:.2e}")
            assert ok(r)
            assert err <= tol
        u, r = c.evaluate(family, yd, sd, yd, xi, rc, tol, report=True)
        assert (r.M, r.P, r.Pg, r.Mt) == (r0.M, r0.P, r0.Pg, r0.Mt)
    finally:
        c.close()


def test_forced_plan_parameters_out_of_range():
    y, s, yd, sd, xi, rc = _problem("stokeslet", 300, 78)
    c = ehs.Context(0)
    try:
        c.set_option(ehs.OPT_PRECISION, 1)
        for opt, val, reset in ((ehs.OPT_FORCE_P, 31, 0), (ehs.OPT_FORCE_P, 13, 0), (ehs.OPT_FORCE_MT, 101, 0),
                                (ehs.OPT_GATHER_EXTRA, 3, -1)):
            c.set_option(opt, val)
            with pytest.raises(ehs.EhsError) as e:
                c.evaluate("stokeslet", yd, sd, yd, xi, rc, 1e-10)
            c.set_option(opt, reset)
            assert e.value.code in (ehs.EHS_EINVAL, ehs.EHS_ERANGE)
        c.evaluate("stokeslet", yd, sd, yd, xi, rc, 1e-10)
    finally:
        c.close()
