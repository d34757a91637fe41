"""Learned Newton guess on the GPU: the MFMA training kernels against the FP64
numpy reference (same BF16-rounded weights and inputs), harvest parity with
the oracle, invariance of the answer under the learned guess, and the
iteration-count report (previous-step W vs learned vs cold start)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import mlp_oracle as M  # noqa: E402
from paper_2401_03008_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu
VA = I.cpa_alfven_speed()
SCALE = [1.0, VA, VA, VA, 1.0, 1.0, 1.0, 1.0]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)


def _mlp(seed=0):
    from paper_2401_03008_amd.learned import Mlp
    return Mlp(seed=seed)


def _ref_theta(mlp):
    """FP64 parameters as the kernels see them: BF16 weights, FP32 biases."""
    p = mlp.params.double().cpu().numpy()
    w = mlp.w.float().double().cpu().numpy()
    th = w.copy()
    for o, n in ((320, 64), (4480, 64), (4672, 2)):
        th[o:o + n] = p[o:o + n]
    return th


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("batch", [1000, 4096, 37])
def test_forward_matches_reference(batch):
    mlp = _mlp(3)
    rng = np.random.default_rng(batch)
    x = rng.normal(size=(batch, 5)).astype(np.float32)
    y = mlp.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    th = _ref_theta(mlp)
    xr = M.bf16_round(x.astype(np.float64))
    yr, _ = M.forward(th, xr)
    assert _rel_l2(y, yr) < 2e-2
    # emulating the BF16 rounding of the hidden activations gives ~FP32 agreement
    p = M.unpack(th)
    h1 = M.bf16_round(np.maximum(xr @ p["W1"].T + p["b1"], 0))
    h2 = M.bf16_round(np.maximum(h1 @ p["W2"].T + p["b2"], 0))
    ye = h2 @ p["W3"].T + p["b3"]
    assert _rel_l2(y, ye) < 2e-3


def test_backward_matches_reference():
    """GPU gradients vs the CPU FP64 gradients on identical BF16-rounded
    weights and inputs: relative L2 <= 2e-2 overall and per tensor."""
    mlp = _mlp(4)
    rng = np.random.default_rng(9)
    B = 2000
    x = rng.normal(size=(B, 5)).astype(np.float32)
    t = rng.normal(size=(B, 2)).astype(np.float32)
    loss = mlp.loss_and_grad(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"))
    g = mlp.grad.double().cpu().numpy()
    th = _ref_theta(mlp)
    xr = M.bf16_round(x.astype(np.float64))
    yr, cache = M.forward(th, xr)
    gr = M.backward(th, cache, M.loss_grad(yr, t.astype(np.float64)))
    assert loss.item() == pytest.approx(M.loss(yr, t.astype(np.float64)), rel=2e-2)
    assert _rel_l2(g, gr) < 2e-2
    for name, _ in M.SHAPES:
        o = M.unpack(np.arange(M.NPARAM))[name].ravel().astype(int)
        assert _rel_l2(g[o], gr[o]) < 3e-2, name


def test_adam_matches_reference():
    mlp = _mlp(5)
    rng = np.random.default_rng(2)
    g = rng.normal(size=M.NPARAM).astype(np.float32)
    p0 = mlp.params.double().cpu().numpy()
    mlp.grad.copy_(torch.tensor(g, device="cuda"))
    mlp.adam_step(lr=1e-3)
    mlp.grad.copy_(torch.tensor(0.5 * g, device="cuda"))
    mlp.adam_step(lr=1e-3)
    th, m, v = M.adam(p0, np.zeros(M.NPARAM), np.zeros(M.NPARAM), g.astype(np.float64), 1)
    th, m, v = M.adam(th, m, v, 0.5 * g.astype(np.float64), 2)
    np.testing.assert_allclose(mlp.params.double().cpu().numpy(), th, rtol=0, atol=1e-6)
    np.testing.assert_array_equal(mlp.w.float().cpu().numpy(),
                                  M.bf16_round(mlp.params.double().cpu().numpy()).astype(np.float32))


def test_harvest_matches_oracle():
    """Every cell harvested (frac = 1) on a ragged turbulence box: the set of
    (features, targets) equals the oracle's, compared after sorting."""
    from paper_2401_03008_amd.solver import Solver
    shape = (12, 20, 40)
    prim5, bf = I.turbulence((40, 20, 12), gamma_max=2.0)
    S = Solver(40, 20, 12)
    S.init(prim5, bf)
    f, t = S.harvest(40 * 20 * 12, 1.0, seed=5)
    f, t = f.double().cpu().numpy(), t.double().cpu().numpy()
    S.close()
    assert f.shape[0] == 40 * 20 * 12
    g = O.Grid(40, 20, 12)
    cons, W = g.init(prim5, bf)
    prim, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    D, U = cons[0].ravel(), cons[4].ravel()
    S3 = np.stack([c.ravel() for c in cons[1:4]], 1)
    B3 = np.stack([prim[5 + d].ravel() for d in range(3)], 1)
    fr = M.features(D, S3, U, B3)
    tr = M.targets(prim[0].ravel(), np.stack([prim[1 + d].ravel() for d in range(3)], 1),
                   prim[4].ravel())
    from scipy.spatial import cKDTree
    A = np.concatenate([f, t], 1)
    R = np.concatenate([fr, tr], 1)
    # match each harvested row to its nearest oracle row (output order is
    # arbitrary); the rows are FP32 copies of FP64 values
    dist, idx = cKDTree(R).query(A)
    assert len(np.unique(idx)) == len(idx)
    np.testing.assert_allclose(A, R[idx], rtol=2e-6, atol=1e-6)


def _train_on_runs(steps=1500):
    """Pairs harvested from the solver itself: the CPA waves (C1/C2 type) and
    64^3 turbulence at sigma0 = 1, 3, 10, a few steps into each run."""
    from paper_2401_03008_amd.learned import harvest_training_set
    feats, targs = harvest_training_set()
    mlp = _mlp(0)
    hist = mlp.fit(feats, targs, steps=steps, batch=4096, lr=2e-3, seed=1, log_every=250)
    return mlp, feats, targs, hist


def test_training_reduces_loss_and_predicts():
    mlp, feats, targs, hist = _train_on_runs()
    print("[gpu] training loss", hist, "pairs", feats.shape[0], flush=True)
    assert hist[-1][1] < 0.05 * hist[0][1]
    pred = mlp.predict(feats[:4096])
    err = (pred - targs[:4096]).abs().mean(0)
    print("[gpu] mean |error| of (log(p/D), log Gamma):", err.tolist(), flush=True)
    assert float(err.max()) < 0.2


def test_learned_guess_same_answer_cpa():
    """CPA 32^3, 10 steps: learned-guess primitives equal the plain ones to
    1e-12 L1 relative, both with the network where no previous W exists
    (here: every cell after a restart from conserved data alone) and with the
    network first in every cell; random (untrained) weights also give the
    same answer (Newton converges from any usable start), and with a
    4-iteration cap the bad guesses fall back (to U, or to the previous W),
    still with the same answer."""
    from paper_2401_03008_amd.solver import Solver
    mlp, *_ = _train_on_runs(steps=400)
    rnd = _mlp(7)
    prim5, bf, _ = I.cpa(32, diagonal=True)

    def run(guess, net=None, maxit=50, restart=False):
        S = Solver(32, newton_maxit=maxit)
        S.init(prim5, bf)
        if restart:  # conserved data only: no previous W anywhere
            st = S.get_state()
            S.set_state(st["cons"], st["bface"], None, st["t"], st["step"])
        if net is not None:
            S.set_mlp(net)
            S.set_guess(guess)
        S.step(10)
        S.set_guess("prev")
        P = S.primitives().cpu().numpy()
        d = S.diagnostics(raise_on_error=False)
        S.close()
        return P, d

    P0, d0 = run("prev")
    cases = [("mlp", mlp, 50, True), ("mlp", rnd, 50, True), ("mlp", rnd, 4, True),
             ("mlp_all", mlp, 50, False), ("mlp_all", rnd, 50, False), ("mlp_all", rnd, 4, False)]
    for guess, net, maxit, restart in cases:
        P1, d1 = run(guess, net, maxit, restart)
        assert d1["c2p_failures"] == 0 and d1["rc"] == 0
        for q in range(8):
            a = np.abs(P1[q] - P0[q]).sum() / max(np.abs(P0[q]).sum(), P0[q].size * SCALE[q])
            assert a <= 1e-12, (q, a, guess, maxit)
        if maxit == 4:
            assert d1["mlp_fallbacks"] > 0, guess


def _iteration_rows(S):
    d = S.diagnostics(raise_on_error=False)
    h = np.array(d["newton_hist"], dtype=np.float64)
    cdf = np.cumsum(h) / h.sum()
    return {"mean_iters": d["newton_iters"] / d["newton_calls"],
            "p50": int(np.searchsorted(cdf, 0.5)), "p99": int(np.searchsorted(cdf, 0.99)),
            "fallback_rate": d["mlp_fallbacks"] / d["newton_calls"],
            "failures": d["c2p_failures"], "hist": d["newton_hist"]}


def test_iteration_report_turbulence():
    """The gain report on the turbulence set-up (C4 type, 128^3, sigma0 = 10,
    Gamma up to 5), measured from the same state over the same steps.

    Warm (4 steps from a state with the previous W): the previous-step W,
    the learned guess where no usable previous W exists (so the previous W
    everywhere here: the same iterations as the plain form, cell for cell),
    the network first in every cell, and a cold start (W0 = U).  The
    measured relation: the previous W is the best start (the network's guess
    is further from the root), so the network first costs iterations.

    Restart (the inversion of the conserved state alone, no W): the method
    without the network starts from U; the network cuts that by a quarter or
    more.  All answers equal the plain one's to 1e-10."""
    from paper_2401_03008_amd.solver import Solver
    mlp, *_ = _train_on_runs()
    n = 128
    prim5, bf = I.turbulence(n, sigma0=10.0, gamma_max=5.0, device="cuda")
    rows, prims = {}, {}
    for guess in ("prev", "mlp", "mlp_all", "cold"):
        S = Solver(n, pfloor=1e-10)
        S.init(prim5, bf)
        S.step(2)
        S.set_mlp(mlp)
        S.set_guess(guess)
        S.reset_counters()
        S.kernel_timing(True)
        S.step(4)
        kt = S.kernel_times()
        rows[guess] = _iteration_rows(S)
        rows[guess]["c2p_ms"] = kt["c2p"][0] / max(kt["c2p"][1], 1)
        S.set_guess("prev")
        prims[guess] = S.primitives()
        S.close()
    for guess in ("prev", "mlp"):
        S = Solver(n, pfloor=1e-10)
        S.init(prim5, bf)
        S.step(2)
        st = S.get_state()
        S.set_state(st["cons"], st["bface"], None, st["t"], st["step"])
        S.set_mlp(mlp)
        S.set_guess(guess)
        S.reset_counters()
        prims["restart_" + guess] = S.primitives()  # one inversion of every cell
        rows["restart_" + guess] = _iteration_rows(S)
        S.close()
    print("[gpu] Newton iterations (turbulence 128^3):",
          {k: {m: v for m, v in r.items() if m != "hist"} for k, r in rows.items()}, flush=True)
    for g in rows:
        assert rows[g]["failures"] == 0
    for g in ("mlp", "mlp_all", "cold"):
        a = (prims[g] - prims["prev"]).abs().sum().item() / prims["prev"].abs().sum().item()
        assert a < 1e-10, g
    a = (prims["restart_mlp"] - prims["restart_prev"]).abs().sum().item() / \
        prims["restart_prev"].abs().sum().item()
    assert a < 1e-10
    # warm: the learned form takes the previous W wherever it is usable, in
    # the previous-W kernels (no inference once every cell has a W)
    assert rows["mlp"]["hist"] == rows["prev"]["hist"]
    assert rows["mlp"]["c2p_ms"] < 1.2 * rows["prev"]["c2p_ms"]
    assert rows["cold"]["mean_iters"] > rows["prev"]["mean_iters"]
    assert rows["mlp_all"]["mean_iters"] >= rows["prev"]["mean_iters"]
    assert rows["mlp_all"]["mean_iters"] < rows["cold"]["mean_iters"]
    assert rows["mlp_all"]["fallback_rate"] < 0.01
    # restart: what the trained network gains over the start from U
    assert rows["restart_mlp"]["mean_iters"] < 0.75 * rows["restart_prev"]["mean_iters"]
    assert rows["restart_mlp"]["fallback_rate"] < 0.01


def test_turbulence_run_driver_small():
    """The long-run driver at 64^3: mixed + learned against plain FP64 over
    20 steps -- same answer to the mixed form's precision, div B at round-off,
    spectra logged."""
    from paper_2401_03008_amd.learned import Mlp
    from paper_2401_03008_amd.runs import compare_runs, turbulence_run
    mlp, *_ = _train_on_runs(steps=300)
    a = turbulence_run(64, 20, precision="fp64", log_every=10, spectrum_every=10)
    b = turbulence_run(64, 20, precision="mixed", mlp=mlp, log_every=10, spectrum_every=10)
    assert "error" not in a and "error" not in b
    assert max(x[2] for x in a["divb"]) < 1e-11 and max(x[2] for x in b["divb"]) < 1e-11
    assert len(a["spectra"]) == 3 and len(a["spectra"][0]["E_v"]) == 31  # steps 0, 10, 20
    diff = compare_runs(b, a)
    print("[gpu] mixed+learned vs fp64 (64^3 turbulence, 20 steps):", ["%.1e" % d for d in diff],
          "newton", a["newton"], b["newton"], flush=True)
    assert max(diff) < 1e-4


def test_in_kernel_guess_matches_reference():
    """The learned guess as the inversion kernel computes it (srmhd_mlp_guess:
    the same feature and in-wavefront MFMA inference code) against the FP64
    reference network on the same BF16-rounded weights, on a ragged
    turbulence box (x rows shorter than a wavefront, partial tiles in y).
    Features come from the oracle's inversion inputs (conserved D, S, U and
    centred B), standardised with the network's normalisation."""
    from paper_2401_03008_amd.solver import Solver
    nx, ny, nz = 40, 10, 7
    prim5, bf = I.turbulence((nx, ny, nz), sigma0=3.0, gamma_max=3.0)
    mlp = _mlp(6)
    g = O.Grid(nx, ny, nz)
    cons, W = g.init(prim5, bf)
    prim, _, nf = g.c2p(cons, bf, W)
    assert nf == 0
    D, U = cons[0].ravel(), cons[4].ravel()
    S3 = np.stack([c.ravel() for c in cons[1:4]], 1)
    B3 = np.stack([prim[5 + d].ravel() for d in range(3)], 1)
    fr = M.features(D, S3, U, B3)
    mlp.norm = [*fr.mean(0), *fr.std(0), -1.0, 0.2, 0.5, 0.3]
    S = Solver(nx, ny, nz)
    S.init(prim5, bf)
    S.set_mlp(mlp)
    W_before = S.W.clone()
    out, w0 = S.mlp_guess()
    torch.cuda.synchronize()
    assert torch.equal(S.W, W_before)  # the probe leaves the state's W alone
    out = out.double().cpu().numpy().reshape(2, -1).T
    w0 = w0.cpu().numpy().ravel()
    S.close()
    nrm = np.array(mlp.norm)
    xr = (fr - nrm[0:5]) / nrm[5:10]
    th = _ref_theta(mlp)
    yr, _ = M.forward(th, M.bf16_round(xr))
    ref = yr * nrm[12:14] + nrm[10:12]
    assert out.shape == ref.shape == (nx * ny * nz, 2)
    assert np.isfinite(out).all()
    assert _rel_l2(out, ref) < 2e-2
    # with the BF16 rounding of the hidden activations emulated as well
    p = M.unpack(th)
    h1 = M.bf16_round(np.maximum(M.bf16_round(xr) @ p["W1"].T + p["b1"], 0))
    h2 = M.bf16_round(np.maximum(h1 @ p["W2"].T + p["b2"], 0))
    ye = (h2 @ p["W3"].T + p["b3"]) * nrm[12:14] + nrm[10:12]
    print(f"[gpu] in-kernel guess: rel L2 {_rel_l2(out, ref):.2e} (FP64), "
          f"{_rel_l2(out, ye):.2e} (BF16 activations)", flush=True)
    assert _rel_l2(out, ye) < 5e-3
    # W0 from the outputs: D Gamma + 4 p Gamma^2 (gamma 4/3), log Gamma >= 0
    lor = np.exp(np.maximum(out[:, 1], 0.0))
    pg = D * np.exp(out[:, 0])
    np.testing.assert_allclose(w0, D * lor + 4.0 * pg * lor * lor, rtol=2e-6)
