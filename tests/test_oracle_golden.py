"""The oracle against values the paper prints (fixtures under tests/golden,
each citing its passage)."""
import os

import numpy as np
import pytest

from oracle import basis, hermite, mg, sipg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _blocks(name):
    out, cur = {}, None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.isalpha():
            cur = out.setdefault(line, [])
        else:
            cur.append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def _keys(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.mark.parametrize("p,h", [(3, 0.37), (5, 0.2)])
def test_hermite_face_stencil_as_printed(p, h):
    """The four coupling blocks built from the Hermite-type basis' own
    endpoint data, restricted to the two layers on each side, are the
    printed stencil."""
    g = _blocks("hermite_face_stencil.txt")
    sigma, beta = 11.0, 1.0 / (2 * h)
    printed = sigma * g["sigma"] + beta * g["beta"]
    e0, g0, e1, g1 = hermite.endpoint_vectors(p)
    N = basis.face_blocks(e0, g0 / h, e1, g1 / h, sigma)
    minus, plus = [p, p - 1], [0, 1]
    got = np.block([[N["--"][np.ix_(minus, minus)], N["-+"][np.ix_(minus, plus)]],
                    [N["+-"][np.ix_(plus, minus)], N["++"][np.ix_(plus, plus)]]])
    assert np.allclose(got, printed, atol=1e-10 * sigma)


def test_mg_pcg_configuration_and_iterations_as_reported():
    """The oracle's solver in the printed configuration: the Chebyshev
    interval and degree, a one-cell coarsest level of 64 unknowns at p = 3,
    and the iteration count of the printed range (a random right-hand side
    on a 4^3 cube stands in for the paper's problem; one iteration either
    way is allowed for that)."""
    c = _keys("mg_pcg_configuration.txt")
    p = int(c["degree"])
    assert mg.INTERVAL == (c["interval_low"], c["interval_high"])
    assert len(mg.chebyshev_weights()) == int(c["chebyshev_degree"])
    m = 4
    H = mg.Hierarchy(p, m, C=c["penalty_C"])
    assert H.A[-1].shape[0] == int(c["coarse_unknowns"])
    b = np.random.default_rng(0).uniform(-1, 1, m ** 3 * (p + 1) ** 3)
    _, it, _ = sipg.pcg(H.A[0], b, H.vcycle, c["rtol"], 100, criterion="preconditioned")
    assert c["iterations_min"] - 1 <= it <= c["iterations_max"] + 1
