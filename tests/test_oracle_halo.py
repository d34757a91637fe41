"""The periodic box split into z-slabs with ghost planes and one exchange per
Runge-Kutta stage (the enlarged halo the paper proposes in its closing
section for its MPI decomposition), on the CPU oracle: bit for bit the
undivided run when the ghost depth covers one stage's stencils (4 planes; 8
with HO), and not with one plane less, which pins the derived depth."""
import numpy as np
import pytest

import oracle as O
from oracle.slabs import SlabRun, ghost_depth
from paper_2401_03008_amd import inputs as I


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


def _undivided(n, prim5, bf, steps, **kw):
    g = O.Grid(n, **kw)
    cons, W = g.init(prim5, bf)
    bfo = [b.copy() for b in bf]
    t, dt, nfail = g.step(cons, bfo, W, steps)
    assert nfail == 0
    return cons, bfo, W, t


def _split(n, prim5, bf, steps, bounds, ghost, **kw):
    g = O.Grid(n, **kw)
    cons, W = g.init(prim5, bf)
    run = SlabRun(n, bounds, ghost, **kw)
    run.set_state(cons, [b.copy() for b in bf], W)
    run.step(steps)
    c, b, w = run.state()
    return c, b, w, run.t


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


CASES = [
    # (label, initial data, slab heights, scheme)
    ("cpa-diag", "cpa", [16, 16], {}),
    ("turb-3slabs-llf", "turb", [10, 12, 10], {"riemann": 1, "pfloor": 1e-10}),
    ("cpa-mc-rk2", "cpa", [8, 24], {"recon": 1, "time_order": 2}),
    ("cpa-ho", "cpa", [16, 16], {"ho": 1}),
]


def _data(kind, n):
    if kind == "cpa":
        prim5, bf, _ = I.cpa(n, diagonal=True)
    else:
        prim5, bf = I.turbulence(n, sigma0=10.0, gamma_max=3.0)
    return prim5, bf


@pytest.mark.parametrize("label,kind,bounds,kw", CASES, ids=[c[0] for c in CASES])
def test_slabs_reproduce_undivided_run_bitwise(label, kind, bounds, kw):
    n, steps = 32, 2
    prim5, bf = _data(kind, n)
    G = ghost_depth(kw.get("ho", 0) == 1)
    ref = _undivided(n, prim5, bf, steps, **kw)
    got = _split(n, prim5, bf, steps, bounds, G, **kw)
    assert _same(got[0], ref[0]), "conserved variables differ"
    assert _same(got[1], ref[1]), "face B differs"
    assert np.array_equal(got[2], ref[2]), "Newton guess W differs"
    assert got[3] == ref[3]


@pytest.mark.parametrize("ho", [0, 1])
def test_one_plane_less_is_not_enough(ho):
    """With G - 1 ghost planes the planes next to each slab edge read
    primitives or faces of a plane the exchange did not fill: the run
    departs from the undivided one."""
    n, steps = 32, 1
    prim5, bf = _data("cpa", n)
    kw = {"ho": ho}
    G = ghost_depth(ho == 1)
    ref = _undivided(n, prim5, bf, steps, **kw)
    got = _split(n, prim5, bf, steps, [16, 16], G - 1, **kw)
    assert not _same(got[0] + got[1], ref[0] + ref[1])


def test_ghost_depth_is_the_stage_dependency():
    """The depth the slabs use is the reach of one stage along z, measured on
    the undivided oracle: perturbing one plane of the state changes L(U) on
    planes up to 3 above and 4 below it (plain), 7 above and 8 below it (HO)
    -- so a plane's update reads planes k-4..k+3 (k-8..k+7)."""
    n = 32
    prim5, bf = _data("turb", n)
    for ho, (below, above) in ((0, (4, 3)), (1, (8, 7))):
        g = O.Grid(n, ho=ho, pfloor=1e-10)
        cons, W = g.init(prim5, bf)
        prim, _, _ = g.c2p(cons, bf, W.copy())
        r0, _ = g.rhs(prim, bf)
        reach = set()
        k0 = 16
        for arrs, idx in ((cons, range(5)), (bf, range(3))):
            for n_ in idx:
                c2 = [a.copy() for a in cons]
                b2 = [a.copy() for a in bf]
                tgt = c2[n_] if arrs is cons else b2[n_]
                tgt[k0] *= 1.0 + 1e-6
                p2, _, _ = g.c2p(c2, b2, W.copy())
                r1, _ = g.rhs(p2, b2)
                for q in range(8):
                    ks = np.nonzero(np.any(r1[q] != r0[q], axis=(1, 2)))[0]
                    reach.update(int(k) - k0 for k in ks)
        assert min(reach) == -above and max(reach) == below, (ho, sorted(reach))
        assert ghost_depth(ho == 1) == max(below, above)
