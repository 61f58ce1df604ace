"""The allocation-free entry point, ewald_halfspace_noalloc, against the
existing entry points ewald_halfspace_{stokeslet,stresslet,rotlet}.

Both run the same kernels under the same plan (the allocation-free call may
use smaller slab groups of the transform pipeline, which does not change the
arithmetic), so the results agree to rounding; both are also held to the
oracle at tol.  Two calls in a row, the second with a smaller input and a
different grid size, so that the second finds the first's octants and
workspace contents in the scratch.  Device memory does not change over the
allocation-free calls, and a problem larger than the scratch is refused.
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


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("fam,prec", [("stokeslet", 1), ("rotlet", 1), ("stresslet", 1), ("stokeslet", 2)])
def test_noalloc_matches_the_allocating_entry_point(fam, prec):
    tol = 1e-10 if prec == 1 else 1e-5
    ctx = ehs.Context(0)
    try:
        ctx.set_option(ehs.OPT_PRECISION, prec)
        cases = []
        for n, seed in ((1000, 71), (400, 72)):  # the second smaller, on another grid size
            y, s = workloads.make(fam, n, seed)
            rc = _rc(300, n)
            xi = ehs.xi_for_cutoff(fam, rc, tol / 2)
            yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
            out = torch.full((n, 3), float("nan"), dtype=torch.float64, device=DEV)
            cases.append((n, y, s, yd, sd, xi, rc, out))
        refs = [ctx.evaluate(fam, yd, sd, yd, xi, rc, tol).cpu().numpy() for n, y, s, yd, sd, xi, rc, _ in cases]
        before = _free()
        reps = []
        for n, y, s, yd, sd, xi, rc, out in cases:
            _, rep = ctx.evaluate_noalloc(fam, yd, sd, yd, xi, rc, tol, out, report=True)
            reps.append(rep)
        after = _free()
        print(f"{fam} prec={prec}: device memory change over the calls {(before - after) / 2**20:.2f} MiB")
        assert before - after < 32 * 2**20
        assert reps[0].Mt != reps[1].Mt
        for (n, y, s, yd, sd, xi, rc, out), ref, rep in zip(cases, refs, reps):
            got = out.cpu().numpy()
            diff = oracle.rel_rms(ref, got)
            err = oracle.rel_rms(oracle.halfspace(fam, y, s, y), got)
            print(f"  N={n} Mt={rep.Mt} zslab={rep.zslab} precision={rep.precision}: "
                  f"vs entry point {diff:.2e}, vs oracle {err:.2e}")
            assert rep.precision == prec
            assert np.all(np.isfinite(got))
            assert diff <= 1e-13
            assert err <= tol
    finally:
        ctx.close()


def test_noalloc_refuses_a_problem_larger_than_its_scratch():
    ctx = ehs.Context(0)
    try:
        ctx.set_option(ehs.OPT_PRECISION, 1)
        n = 20_000
        y, s = workloads.make("stresslet", n, 73)
        rc = _rc(300, n)
        xi = ehs.xi_for_cutoff("stresslet", rc, 0.5e-10)
        yd, sd = torch.from_numpy(y).to(DEV), torch.from_numpy(s).to(DEV)
        out = torch.empty((n, 3), dtype=torch.float64, device=DEV)
        with pytest.raises(ehs.EhsError) as e:
            ctx.evaluate_noalloc("stresslet", yd, sd, yd, xi, rc, 1e-10, out)
        assert e.value.code == ehs.EHS_ETOOBIG
        # a small problem still runs afterwards
        y, f = workloads.uniform_stokeslet(500, 74)
        yd, fd = torch.from_numpy(y).to(DEV), torch.from_numpy(f).to(DEV)
        rc = _rc(300, 500)
        xi = ehs.xi_for_cutoff("stokeslet", rc, 0.5e-10)
        out = torch.empty((500, 3), dtype=torch.float64, device=DEV)
        ctx.evaluate_noalloc("stokeslet", yd, fd, yd, xi, rc, 1e-10, out)
        assert oracle.rel_rms(oracle.halfspace("stokeslet", y, f, y), out.cpu().numpy()) <= 1e-10
    finally:
        ctx.close()
