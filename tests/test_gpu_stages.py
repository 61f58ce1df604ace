"""Stage-level checks of the GPU path, so that a failure names its stage.

The real-space sum's cell lists (Sec. 4 and 5.1: pairs within r_c only) are
checked by count: the kernels count the (target, source) pairs they
evaluate (direct pairs with 0 < |x - y| < r_c, image pairs with
|x - y^I| < r_c, y^I = (y1, y2, -y3)), which must equal a brute-force count
over all pairs, for every cell reach and for point sets uniform and
clustered at the wall, with the targets the sources or separate.  A cell
walk that misses a neighbour cell, or visits one twice, changes the count.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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
