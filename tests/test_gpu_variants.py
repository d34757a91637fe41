"""GPU parity of the scheme variants against the oracle: HO = YES (sixth-order
INT and DER, point-value MP5), linear MC reconstruction, SSP-RK2, on the same
seeded inputs and with the bars of the plain path (rough states: L1 <= 1e-10,
element-wise 1e-9 of max |L(U)|; smooth waves: L1 <= 1e-12 per variable)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2401_03008_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

VA = I.cpa_alfven_speed()
SCALE = [1.0, VA, VA, VA, 1.0, 1.0, 1.0, 1.0]
VARIANTS = {
    "ho": (dict(high_order=True), dict(ho=1)),
    "mc": (dict(recon="mc"), dict(recon=1)),
    "mc_rk2": (dict(recon="mc", time_order=2), dict(recon=1, time_order=2)),
    "ho_rk2": (dict(high_order=True, time_order=2), dict(ho=1, time_order=2)),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)


def _solver(shape, **kw):
    from paper_2401_03008_amd.solver import Solver
    nz, ny, nx = shape
    print(f"[gpu] Solver {nx}x{ny}x{nz} {kw}", flush=True)
    return Solver(nx, ny, nz, **kw)


def _oracle(shape, **kw):
    nz, ny, nx = shape
    return O.Grid(nx, ny, nz, **kw)


def l1rel(a, b, s):
    return np.abs(a - b).sum() / max(np.abs(b).sum(), a.size * s)


def _rough_state(shape, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, shape)
    p = rng.uniform(0.1, 1.0, shape)
    d = rng.normal(size=(3,) + shape)
    d /= np.linalg.norm(d, axis=0)
    v = d * rng.uniform(0.0, 0.99, shape)
    bf = [np.ascontiguousarray(rng.normal(size=shape)) for _ in range(3)]
    return [np.ascontiguousarray(a) for a in (rho, v[0], v[1], v[2], p)], bf


@pytest.mark.parametrize("variant", ["ho", "mc"])
@pytest.mark.parametrize("shape,seed", [((12, 20, 72), 13), ((9, 10, 11), 15), ((21, 18, 66), 16)])
def test_rhs_rough_state(variant, shape, seed):
    """L(U) element by element on rough random states (ragged tiles, every
    limiter branch, first-order fallbacks); amax exactly.  The bound is the
    rough-state bound of the plain path (same conditioning argument)."""
    gkw, okw = VARIANTS[variant]
    prim5, bf = _rough_state(shape, seed)
    S = _solver(shape, **gkw)
    S.init(prim5, bf)
    R, amax = S.rhs()
    torch.cuda.synchronize()
    R = R.cpu().numpy()
    d = S.diagnostics()
    S.close()
    g = _oracle(shape, **okw)
    cons, W = g.init(prim5, bf)
    Pr, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    Rr, amax_r = g.rhs(Pr, bf)
    assert d["recon_fallbacks"] == g.stats.recon_fallbacks
    assert amax.item() == pytest.approx(amax_r, rel=1e-13)
    for q in range(8):
        scale = np.abs(Rr[q]).max()
        assert np.abs(R[q] - Rr[q]).sum() / np.abs(Rr[q]).sum() <= 1e-10, q
        np.testing.assert_allclose(R[q], Rr[q], rtol=0, atol=1e-9 * scale, err_msg=f"comp {q}")


@pytest.mark.parametrize("variant", ["ho", "mc", "mc_rk2", "ho_rk2"])
def test_step_parity_diagonal_wave(variant):
    """Diagonal wave 24^3, 8 steps at CFL 0.5: primitives and face B within
    L1 1e-12 of the oracle; dt agrees; div B (in the variant's own
    differences) stays at round-off."""
    gkw, okw = VARIANTS[variant]
    n = 24
    shape = (n, n, n)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    S = _solver(shape, **gkw)
    S.init(prim5, bf)
    S.step(8)
    P = S.primitives().cpu().numpy()
    t, st, dt = S.time()
    d = S.diagnostics()
    Bg = S.bface.cpu().numpy()
    S.close()
    g = _oracle(shape, **okw)
    cons, W = g.init(prim5, bf)
    bfo = [b.copy() for b in bf]
    tr, dtr, nf = g.step(cons, bfo, W, 8)
    Pr, _, _ = g.c2p(cons, bfo, W)
    assert st == 8 and nf == 0 and d["c2p_failures"] == 0
    assert dt == pytest.approx(dtr, rel=1e-13)
    assert t == pytest.approx(tr, rel=1e-13)
    for q in range(8):
        assert l1rel(P[q], Pr[q], SCALE[q]) <= 1e-12, (variant, q)
    for k in range(3):
        assert l1rel(Bg[k], bfo[k], 1.0) <= 1e-12
    assert d["divb_max"] / n < 1e-11
    assert d["divb_max"] == pytest.approx(g.divb_max(bfo), rel=1e-6, abs=1e-12 * n)


def test_ho_divb_of_rough_field_is_kept():
    """HO on a rough, non-solenoidal face field (small perturbation of the
    wave): the HO divergence is not small, but the HO curl keeps it: its
    maximum after 3 steps equals the initial one to round-off, and equals
    the oracle's."""
    n = 16
    shape = (n, n, n)
    rng = np.random.default_rng(21)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    bf = [np.ascontiguousarray(b + 1e-3 * rng.normal(size=shape)) for b in bf]
    S = _solver(shape, high_order=True)
    S.init(prim5, bf)
    d0 = S.diagnostics()["divb_max"]
    S.step(3)
    d1 = S.diagnostics()
    S.close()
    g = _oracle(shape, ho=1)
    assert d0 == pytest.approx(g.divb_max(bf), rel=1e-12)
    assert d0 > 0.01  # the perturbation's divergence, ~1e-3 x 1.7 x n per direction
    assert d1["c2p_failures"] == 0
    assert abs(d1["divb_max"] - d0) <= 1e-9 * d0


def test_ho_sampled_cells_256():
    """HO at 256^3 in the benchmark's launch shape: L(U) on 512 sampled
    cells (box corners included) against the oracle's per-cell evaluation."""
    n = 256
    prim5, bf, _ = I.cpa(n, diagonal=True)
    S = _solver((n, n, n), high_order=True)
    S.init(prim5, bf)
    R, _ = S.rhs()
    R = R.reshape(8, -1)
    rng = np.random.default_rng(2560)
    cells = np.unique(np.concatenate([rng.choice(n ** 3, 506, replace=False),
                                      [0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n, (n - 1) * n * n]]))
    Rg = R[:, torch.as_tensor(cells, device=R.device)].cpu().numpy().T
    S.close()
    g = O.Grid(n, ho=1)
    cons, W = g.init(prim5, bf)
    Pr, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    Rr = g.rhs_cells(Pr, bf, cells)
    for q in range(8):
        tol = 1e-12 * max(np.abs(Rr[:, q]).max(), float(n))
        np.testing.assert_allclose(Rg[:, q], Rr[:, q], rtol=0, atol=tol)


def test_mixed_ho_close_to_fp64_ho():
    """The mixed form with HO: FP32 REC and fluxes, FP64 elsewhere; after 4
    steps of the 32^3 diagonal wave its primitives are within 1e-5 (L1
    relative) of the FP64 HO run's."""
    n = 32
    shape = (n, n, n)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    out = {}
    for prec in ("fp64", "mixed"):
        S = _solver(shape, high_order=True, precision=prec, dt_fixed=0.2 / n)
        S.init(prim5, bf)
        S.step(4)
        out[prec] = S.primitives().cpu().numpy()
        S.close()
    for q in range(8):
        assert l1rel(out["mixed"][q], out["fp64"][q], SCALE[q]) <= 1e-5, q


@pytest.mark.parametrize("shape,kw,okw", [((2, 3, 20), dict(), dict()),
                                          ((1, 5, 70), dict(high_order=True), dict(ho=1)),
                                          ((3, 1, 9), dict(recon="mc"), dict(recon=1)),
                                          ((9, 2, 20), dict(high_order=True), dict(ho=1))])
def test_rhs_thin_boxes(shape, kw, okw):
    """Directions with fewer than 4 cells (stencils that wrap more than once)
    on rough random states, against the oracle element by element."""
    prim5, bf = _rough_state(shape, 31)
    S = _solver(shape, **kw)
    S.init(prim5, bf)
    R, amax = S.rhs()
    R = R.cpu().numpy()
    S.close()
    g = _oracle(shape, **okw)
    cons, W = g.init(prim5, bf)
    Pr, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    Rr, amax_r = g.rhs(Pr, bf)
    assert amax.item() == pytest.approx(amax_r, rel=1e-13)
    for q in range(8):
        scale = max(np.abs(Rr[q]).max(), 1e-300)
        np.testing.assert_allclose(R[q], Rr[q], rtol=0, atol=1e-9 * scale, err_msg=f"comp {q}")


@pytest.mark.parametrize("kw,okw", [(dict(high_order=True), dict(ho=1)), (dict(), dict())])
def test_2d_turbulence_step_parity(kw, okw):
    """The 2D set-up of Sec. 5 on a 48 x 48 x 1 box, 5 steps: primitives and
    face B within L1 1e-12 of the oracle (velocity scale v_A/4, field scale
    B0/4 for the fluctuating components).  The initial B is the second-order
    discrete curl of a potential: its plain divergence is round-off, its HO
    divergence is truncation-sized; each scheme keeps its own divergence
    unchanged to round-off."""
    n = 48
    prim5, bf, L = I.turbulence2d(n)
    shape = (1, n, n)
    S = _solver(shape, L=L, **kw)
    S.init(prim5, bf)
    div0 = S.diagnostics()["divb_max"]
    S.step(5)
    P = S.primitives().cpu().numpy()
    d = S.diagnostics()
    Bg = S.bface.cpu().numpy()
    S.close()
    g = O.Grid(n, n, 1, lx=L[0], ly=L[1], lz=L[2], **okw)
    cons, W = g.init(prim5, bf)
    bfo = [b.copy() for b in bf]
    _, _, nf = g.step(cons, bfo, W, 5)
    Pr, _, _ = g.c2p(cons, bfo, W)
    assert nf == 0 and d["c2p_failures"] == 0
    va = 10.0 / np.sqrt(301.0)
    sc = [1.0, va / 4, va / 4, va / 4, 50.0, 2.5, 2.5, 10.0]
    for q in range(8):
        assert l1rel(P[q], Pr[q], sc[q]) <= 1e-12, q
    for k in range(3):
        assert l1rel(Bg[k], bfo[k], sc[5 + k]) <= 1e-12
    dx = L[0] / n
    assert abs(d["divb_max"] - div0) * dx < 1e-11
    if not okw.get("ho"):
        assert d["divb_max"] * dx < 1e-11


@pytest.mark.parametrize("kw", [dict(), dict(high_order=True),
                                dict(high_order=True, precision="mixed")])
def test_z_uniform_box_matches_one_cell_deep_bitwise(kw):
    """z-uniform data on a 48 x 48 x 1 box (the unstaged z flux pass, E_x and
    E_y, and the one-plane HO update) and the same data replicated to
    48 x 48 x 8 (their LDS-staged forms on z-deep tiles): every z difference
    is exactly zero and every other operation is the same, so after 3 steps
    each plane of the deep box equals the one-plane box bit for bit -- except
    that with HO the two boxes use two different update kernels, which the
    compiler may contract into FMAs differently; a last-bit difference then
    passes through the Newton inversion (tolerance 1e-14 of W) and the
    cancellation in p, and the planes agree to round-off: measured 1.0e-13
    (FP64) and 7.8e-14 (mixed) of each field's maximum, required <= 1e-12, the
    parity bar; a stencil or staging error shows at 1e-3 and up."""
    n = 48
    prim5, bf, L = I.turbulence2d(n)
    out = {}
    for nz in (1, 8):
        p = [np.ascontiguousarray(np.repeat(a, nz, axis=0)) for a in prim5]
        b = [np.ascontiguousarray(np.repeat(a, nz, axis=0)) for a in bf]
        S = _solver((nz, n, n), L=(L[0], L[1], L[2] * nz), dt_fixed=0.01, **kw)
        S.init(p, b)
        S.step(3)
        out[nz] = (S.primitives().cpu().numpy(), S.bface.cpu().numpy())
        S.close()
    P1, B1 = out[1]
    P8, B8 = out[8]
    worst = 0.0
    for k in range(8):
        for X, Y in ((P8[:, k], P1[:, 0]), (B8[:, k], B1[:, 0])):
            for q in range(X.shape[0]):
                d = np.abs(X[q] - Y[q]).max() / max(np.abs(Y[q]).max(), 1e-300)
                worst = max(worst, d)
    print(f"[gpu] z-uniform deep vs one-plane box, max relative difference: {worst:.2e}", flush=True)
    if kw.get("high_order"):
        assert worst <= 1e-12
    else:
        assert worst == 0.0


def test_llf_with_ho_and_zero_steps():
    """LLF fluxes with HO against the oracle (24^3 diagonal wave, 4 steps),
    and step(0) leaving the state, time and step count untouched."""
    n = 24
    shape = (n, n, n)
    prim5, bf, _ = I.cpa(n, diagonal=True)
    S = _solver(shape, high_order=True, riemann="llf")
    S.init(prim5, bf)
    c0 = S.cons.clone()
    S.step(0)
    t0, st0, _ = S.time()
    assert st0 == 0 and t0 == 0.0 and torch.equal(S.cons, c0)
    S.step(4)
    P = S.primitives().cpu().numpy()
    S.close()
    g = _oracle(shape, ho=1, riemann=1)
    cons, W = g.init(prim5, bf)
    bfo = [b.copy() for b in bf]
    g.step(cons, bfo, W, 4)
    Pr, _, _ = g.c2p(cons, bfo, W)
    for q in range(8):
        assert l1rel(P[q], Pr[q], SCALE[q]) <= 1e-12, q
