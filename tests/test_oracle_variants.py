"""Pins of the oracle's scheme variants: HO = YES (sixth-order INT and DER,
point-value MP5), linear reconstruction with the MC limiter, and SSP-RK2.

The paper names these variants (Sec. 3: INT and DER go beyond second order
only with HO = YES; the benchmark section: second-order time stepping with
linear reconstruction as the faster configuration) but prints none of their
formulas.  Each test checks the oracle against closed forms, polynomial
exactness, measured convergence orders on the exact wave, or an identity of
the discrete operators; nothing here comes from the GPU path.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2401_03008_amd import inputs as I

GAM = 4.0 / 3.0


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


# ------------------------------------------------------------ point formulas
@pytest.mark.parametrize("s,want", [
    ((0.0, 1.0, 4.0), 2.0),     # slopes 1, 3: min(2, 6, 2) = 2
    ((0.0, 1.0, 1.5), 1.375),   # slopes 1, 0.5: min(2, 1, 0.75) = 0.75
    ((0.0, 1.0, 0.0), 1.0),     # extremum: zero slope
    ((3.0, 1.0, 0.0), 0.25),    # slopes -2, -1: -min(4, 2, 1.5) = -1.5
    ((0.0, 1.0, 2.0), 1.5),     # linear: central slope 1
])
def test_mc_closed_form(s, want):
    """MC(a, b) = sign(a) min(2|a|, 2|b|, |a+b|/2) for ab > 0 (van Leer 1977)."""
    assert O.mc(s) == want


def test_mc_exact_on_lines_and_bounded():
    """Exact on linear data from both sides; on random data every face value
    lies between the two cells that share the face (no new extrema)."""
    for a, b in ((0.3, 1.7), (-2.0, 0.25), (5.0, -3.0)):
        v = [a + b * i for i in range(-1, 3)]  # v_{-1}, v_0, v_1, v_2
        face = a + b * 0.5
        assert O.mc(v[0:3]) == pytest.approx(face, abs=1e-15)
        assert O.mc(v[3:0:-1]) == pytest.approx(face, abs=1e-15)
    rng = np.random.default_rng(4)
    for _ in range(2000):
        v = rng.normal(size=4)
        for f in (O.mc(v[0:3]), O.mc(v[3:0:-1])):
            assert min(v[1], v[2]) - 1e-15 <= f <= max(v[1], v[2]) + 1e-15


def test_mp5_point_interpolates_quartics():
    """The HO REC's unlimited value is the 5-point interpolation at the face:
    exact for polynomials of degree 4 (monotone data, so the limiter accepts
    it); the cell-average MP5 on the same data is not (it returns the face
    value of the function whose cell averages are these point values)."""
    p = lambda x: 1.0 + x + 0.1 * x ** 2 - 0.02 * x ** 3 + 0.003 * x ** 4
    s = [p(x) for x in (-2, -1, 0, 1, 2)]
    assert O.mp5_point(s) == pytest.approx(p(0.5), abs=1e-14)
    # mirrored stencil gives the right-biased value at the same face
    r = [p(x) for x in (3, 2, 1, 0, -1)]
    assert O.mp5_point(r) == pytest.approx(p(0.5), abs=1e-14)
    # the average-based kernel differs by -h^2/24 p'' + O(h^4) at this face
    diff = O.mp5(s) - p(0.5)
    assert diff == pytest.approx(-(0.2 - 0.12 * 0.5 + 0.036 * 0.25) / 24.0, rel=0.15)


def test_mp5_point_fifth_order():
    """On a smooth monotone profile the error of the face value falls by
    about 2^5 per halving of the spacing."""
    errs = []
    for h in (0.2, 0.1, 0.05):
        s = [math.tanh(0.7 + h * m) for m in (-2, -1, 0, 1, 2)]
        errs.append(abs(O.mp5_point(s) - math.tanh(0.7 + 0.5 * h)))
    assert math.log2(errs[0] / errs[1]) > 4.6
    assert math.log2(errs[1] / errs[2]) > 4.8


def test_int_ho_polynomials_and_symbol():
    """Sixth-order centre value: exact for quintics; for cos(kx) the result
    is cos(kx_i) (150 cos(t/2) - 25 cos(3t/2) + 3 cos(5t/2))/128, t = kh."""
    q = lambda x: 0.5 - x + 0.3 * x ** 2 + 0.2 * x ** 3 - 0.05 * x ** 4 + 0.01 * x ** 5
    b = [q(m + 0.5) for m in range(-3, 3)]  # faces at -5/2 .. 5/2
    assert O.int_ho(b) == pytest.approx(q(0.0), abs=1e-14)
    for t in (0.1, 0.7, 2.0):
        x0 = 0.37
        b = [math.cos(x0 + t * (m + 0.5)) for m in range(-3, 3)]
        sym = (150 * math.cos(t / 2) - 25 * math.cos(1.5 * t) + 3 * math.cos(2.5 * t)) / 128
        assert O.int_ho(b) == pytest.approx(math.cos(x0) * sym, abs=1e-15)
    # sixth order: error ratio ~64 per halving of t
    e = [abs(O.int_ho([math.cos(0.37 + t * (m + 0.5)) for m in range(-3, 3)]) - math.cos(0.37))
         for t in (0.4, 0.2)]
    assert math.log2(e[0] / e[1]) > 5.8


def test_der_ho_polynomials_and_symbol():
    """Fhat = f - D2 f/24 + 3 D4 f/640 at two faces: the difference divided
    by h is exact for polynomials of degree 6, and for f = sin(kx) equals
    2 s (1 + s^2/6 + 3 s^4/40) cos(kx_i), s = sin(kh/2)."""
    r = lambda x: 1 - 2 * x + x ** 2 - 0.4 * x ** 3 + 0.1 * x ** 4 + 0.03 * x ** 5 - 0.01 * x ** 6
    dr = lambda x: (-2 + 2 * x - 1.2 * x ** 2 + 0.4 * x ** 3 + 0.15 * x ** 4 - 0.06 * x ** 5)
    f = [r(m + 0.5) for m in range(-3, 3)]
    assert O.der_ho(f) == pytest.approx(dr(0.0), abs=1e-13)
    for t in (0.05, 0.5, 1.5):
        x0 = -0.8
        f = [math.sin(x0 + t * (m + 0.5)) for m in range(-3, 3)]
        s = math.sin(t / 2)
        want = 2 * s * (1 + s * s / 6 + 3 * s ** 4 / 40) * math.cos(x0)
        assert O.der_ho(f) == pytest.approx(want, abs=1e-15)


# ------------------------------------------------------------ the operators
def _cons_exact(n, t):
    """Point values of the conserved variables of the diagonal wave (centre B
    exact) and the face-sampled B."""
    prim5, bf, Bc = I.cpa(n, diagonal=True, t=t)
    pr = np.stack(prim5 + Bc, -1).reshape(-1, 8)
    u = np.array([O.prim2cons(x, GAM) for x in pr]).reshape((n, n, n, 8))
    return [np.ascontiguousarray(u[..., q]) for q in range(5)], bf, prim5


def _dudt_exact(n, tau=1e-3):
    """d/dt of the exact wave's state at t = 0 (fourth-order central
    difference in time of the exact solution)."""
    acc = None
    for s, w in ((-2, 1.0), (-1, -8.0), (1, 8.0), (2, -1.0)):
        c, bf, _ = _cons_exact(n, s * tau)
        a = [w * x for x in c + bf]
        acc = a if acc is None else [p + q for p, q in zip(acc, a)]
    return [a / (12 * tau) for a in acc]


def _operator_error(n, norm, **kw):
    cons, bf, prim5 = _cons_exact(n, 0.0)
    g = O.Grid(n, **kw)
    W = (1.0 + 4.0 * 1.0) / (1.0 - (prim5[1] ** 2 + prim5[2] ** 2 + prim5[3] ** 2))
    prim, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    rhs, _ = g.rhs(prim, bf)
    ex = _dudt_exact(n)
    if norm == "max":
        return max(np.abs(rhs[q] - ex[q]).max() for q in range(8))
    return np.mean([np.abs(rhs[q] - ex[q]).mean() for q in range(8)])


def test_operator_orders_on_diagonal_wave():
    """Truncation error of L(U) against the exact time derivative of the
    diagonal wave at 16^3 and 32^3: fifth order with HO (the order the
    paper attributes to MP5 with HO and DER), second order without HO, and
    about second order (L1) with linear MC reconstruction."""
    e_ho = [_operator_error(n, "max", ho=1) for n in (16, 32)]
    e_plain = [_operator_error(n, "max") for n in (16, 32)]
    e_mc = [_operator_error(n, "l1", recon=1) for n in (16, 32)]
    assert math.log2(e_ho[0] / e_ho[1]) > 4.7
    assert 1.8 < math.log2(e_plain[0] / e_plain[1]) < 2.3
    assert 1.5 < math.log2(e_mc[0] / e_mc[1]) < 2.3
    assert e_ho[1] < 0.01 * e_plain[1]


def test_ho_int_centre_field_sixth_order():
    """HO init: the centred B entering the conserved variables is the
    sixth-order interpolation of the face samples (error ratio ~64)."""
    errs = []
    for n in (16, 32):
        prim5, bf, Bc = I.cpa(n, diagonal=True)
        g = O.Grid(n, ho=1)
        cons, W = g.init(prim5, bf)
        prim, _, nf = g.c2p(cons, bf, W)
        assert nf == 0
        for q in range(5):
            np.testing.assert_allclose(prim[q], prim5[q], rtol=0, atol=1e-12)
        errs.append(max(np.abs(prim[5 + d] - Bc[d]).max() for d in range(3)))
    assert math.log2(errs[0] / errs[1]) > 5.7


def _div_ho(b, dx):
    """sum_d of the corrected differences of the face field along d."""
    out = np.zeros_like(b[0])
    for d in range(3):
        ax = 2 - d
        f = [np.roll(b[d], -(m - 3), axis=ax) for m in range(6)]  # f[m] = b at offset m-3
        out += np.vectorize(lambda *v: O.der_ho(v))(*f) / dx[d]
    return out


def test_ho_curl_keeps_ho_divergence():
    """With HO the curl of the corrected edge fields has zero corrected
    divergence for any state: d/dt div_HO B = 0 to round-off on a rough
    random state with a non-solenoidal B."""
    rng = np.random.default_rng(11)
    n = 8
    shape = (n, n, n)
    prim = [rng.uniform(0.5, 2.0, shape)]
    v = rng.normal(size=(3,) + shape)
    v *= rng.uniform(0.0, 0.9, shape) / np.sqrt((v ** 2).sum(0))
    prim += [np.ascontiguousarray(v[i]) for i in range(3)]
    prim += [rng.uniform(0.1, 1.0, shape)]
    bf = [np.ascontiguousarray(rng.normal(size=shape)) for _ in range(3)]
    g = O.Grid(n, ho=1)
    # centred B by the HO INT, through init + inversion
    cons, W = g.init(prim, bf)
    prim8, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    rhs, _ = g.rhs(prim8, bf)
    dB = rhs[5:8]
    scale = max(np.abs(x).max() for x in dB) * n
    div = _div_ho(dB, [1.0 / n] * 3)
    assert np.abs(div).max() <= 1e-13 * scale
    # and the oracle's HO div B diagnostic is that divergence of the field
    assert g.divb_max(bf) == pytest.approx(np.abs(_div_ho(bf, [1.0 / n] * 3)).max(), rel=1e-12)


def test_ho_step_keeps_div_b_on_wave():
    """HO steps on the diagonal wave keep div_HO B at round-off."""
    n = 12
    g = O.Grid(n, ho=1)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    cons, W = g.init(prim5, bf)
    assert g.divb_max(bf) / n < 1e-12
    _, _, nf = g.step(cons, bf, W, 3)
    assert nf == 0
    assert g.divb_max(bf) / n < 1e-12


@pytest.mark.parametrize("kw", [dict(ho=1), dict(recon=1)])
def test_rhs_cells_matches_grid_rhs_variants(kw):
    """The per-cell evaluation agrees bitwise with the grid operator in the
    HO and MC variants as well."""
    rng = np.random.default_rng(5)
    n = 9
    shape = (n, n, n)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    bf = [np.ascontiguousarray(b + 0.05 * rng.normal(size=shape)) for b in bf]
    g = O.Grid(n, **kw)
    cons, W = g.init(prim5, bf)
    prim, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    rhs, _ = g.rhs(prim, bf)
    cells = np.arange(0, n ** 3, 11)
    out = g.rhs_cells(prim, bf, cells)
    full = np.stack([r.ravel() for r in rhs], axis=1)[cells]
    assert np.array_equal(out, full)


@pytest.mark.parametrize("order,ratio", [(2, 4.0), (3, 8.0)])
def test_time_order_self_convergence(order, ratio):
    """Same grid, dt halved twice, same end time: successive differences
    shrink by 2^order (SSP-RK2: 4, SSP-RK3: 8); a wrong stage weight drops
    the order."""
    n = 16
    sols = []
    for r in (1, 2, 4):
        g = O.Grid(n, dt_fixed=0.02 / n / r, time_order=order)
        prim5, bf, _ = I.cpa(n, diagonal=True)
        cons, W = g.init(prim5, bf)
        _, _, nf = g.step(cons, bf, W, 8 * r)
        assert nf == 0
        sols.append(np.concatenate([c.ravel() for c in cons] + [b.ravel() for b in bf]))
    d1 = np.abs(sols[0] - sols[1]).max()
    d2 = np.abs(sols[1] - sols[2]).max()
    assert d1 / d2 == pytest.approx(ratio, rel=0.03)


def test_rk2_conserves_and_preserves_uniform_state():
    """SSP-RK2 keeps a uniform state exactly and conserves the totals of the
    wave to round-off (periodic box)."""
    n = 8
    g = O.Grid(n, time_order=2)
    prim5 = [np.full((n, n, n), v) for v in (1.0, 0.3, -0.2, 0.1, 0.5)]
    bf = [np.full((n, n, n), v) for v in (0.4, 0.0, -0.7)]
    cons, W = g.init(prim5, bf)
    c0 = [c.copy() for c in cons]
    g.step(cons, bf, W, 2)
    for a, b in zip(cons, c0):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-15)
    g = O.Grid(12, time_order=2)
    prim5, bf, _ = I.cpa(12, diagonal=True)
    cons, W = g.init(prim5, bf)
    s0 = g.sums(cons, bf)
    g.step(cons, bf, W, 3)
    s1 = g.sums(cons, bf)
    for a, b in zip(s0, s1):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b))


@pytest.mark.parametrize("kw", [dict(), dict(ho=1)])
def test_z_uniform_box_equals_replicated(kw):
    """A box one cell deep in z (the 2D set-up of Sec. 5) gives, bitwise, the
    operator of the same z-uniform data on a box four cells deep: the
    stencils wrap onto the single layer exactly as onto identical layers."""
    prim5, bf, L = I.turbulence2d(24)
    g1 = O.Grid(24, 24, 1, lx=L[0], ly=L[1], lz=L[2], **kw)
    cons, W = g1.init(prim5, bf)
    P1, _, nf = g1.c2p(cons, bf, W)
    assert nf == 0
    R1, a1 = g1.rhs(P1, bf)
    rep = lambda a: np.ascontiguousarray(np.repeat(a, 4, axis=0))
    g4 = O.Grid(24, 24, 4, lx=L[0], ly=L[1], lz=4 * L[2], **kw)
    cons4, W4 = g4.init([rep(a) for a in prim5], [rep(b) for b in bf])
    P4, _, _ = g4.c2p(cons4, [rep(b) for b in bf], W4)
    R4, a4 = g4.rhs(P4, [rep(b) for b in bf])
    assert a1 == a4
    for q in range(8):
        for k in range(4):
            assert np.array_equal(R4[q][k], R1[q][0]), (q, k)


def test_turbulence2d_initial_data():
    """Sec. 5 set-up: B0 = 10, p0 = 50, v_A = 10/sqrt(301) ~ 0.576 (the
    paper prints 0.57), <|dv|>/v_A = <|dB|>/B0 = 0.25, div B = 0 to
    round-off, 24 modes with 1 <= |k| <= 4."""
    n = 32
    prim5, bf, L = I.turbulence2d(n)
    va = 10.0 / math.sqrt(301.0)
    assert va == pytest.approx(0.57, abs=0.01)
    assert np.all(prim5[0] == 1.0) and np.all(prim5[4] == 50.0) and np.all(bf[2] == 10.0)
    assert np.mean(np.hypot(prim5[1], prim5[2])) / va == pytest.approx(0.25, rel=1e-12)
    h = L[0] / n
    div = (bf[0] - np.roll(bf[0], 1, axis=2)) / h + (bf[1] - np.roll(bf[1], 1, axis=1)) / h
    assert np.abs(div).max() < 1e-12
    modes = I.turbulence2d_modes()
    assert len(modes) == 24 and all(1 <= math.hypot(*k) <= 4 for k in modes)
