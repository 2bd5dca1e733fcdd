"""GPU modal indicator, features and the learned-indicator network against
the oracle (oracle/indicator.py, oracle/mlp.py), through the C-ABI.

Tolerances: outputs are FP32.  Indicator and features are computed in FP64
and rounded once: 2^-24 relative plus FP64 round-off; the indicator's cut at
alpha = 1e-3 is a decision, compared only away from it.  The network runs in
FP32 with BF16 weights: a 16 + 64 + 64 term chain of FP32 sums, so outputs
agree within 2 * 144 * 2^-24 of the absolute-value propagation of the same
network (|W| |x| + |b| layer by layer).  Gradients are FP32 sums over the
batch (64-sample passes, then the passes): held to 1e-4 of their norm."""
import numpy as np
import pytest

from oracle import indicator as IND
from oracle import mlp as MLP
from workloads import states
from workloads.meshes import workload_mesh, random_mesh

pytestmark = pytest.mark.gpu


def _solver(spec, N, u_fn):
    import paper_2607_06045_amd as P
    s = P.Solver(N)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    u = u_fn(x, y)
    s.upload(u)
    return s, u


CASES = {
    "blast": (lambda: workload_mesh("blast22k"), lambda x, y: states.workload_state("blast22k", x, y)),
    "shear": (lambda: random_mesh(2, 8, 2, 0.3, L=2.0, x0=-1.0, y0=-1.0),
              lambda x, y: states.shear_layer(x, y)),
    "random": (lambda: random_mesh(4, 6, 2, 0.4), lambda x, y: states.random_admissible(x, 5)),
}


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("case", sorted(CASES))
def test_hennemann_and_features_parity(case, N):
    import paper_2607_06045_amd as P
    mesh_fn, u_fn = CASES[case]
    s, u = _solver(mesh_fn(), N, u_fn)
    a = s.indicator(P.IND_HENNEMANN)
    en = IND.hennemann_energy(u, N)
    ref = IND.hennemann(u, N)
    T = IND.threshold(N)
    raw = 1.0 / (1.0 + np.exp(-(np.log(9999.0) / T) * (en - T)))
    away = np.abs(raw - IND.ALPHA_MIN) > 1e-9
    err = np.abs(a - ref)[away].max()
    print(f"{case} N={N}: E={s.E}, alpha>0 on {(ref > 0).sum()}, max|da|={err:.2e}", flush=True)
    assert err <= 2.0 ** -24 * 0.5 + 1e-12
    f = s.features()
    fr = IND.features(u, N)
    assert np.abs(f - fr).max() <= 2.0 ** -24 + 1e-12
    # device outputs are the same values
    import torch
    assert np.array_equal(s.indicator(P.IND_HENNEMANN, device=True).cpu().numpy(), a)
    assert np.array_equal(s.features(device=True).cpu().numpy(), f)


def _abs_scale(w, x):
    p = MLP.unpack(MLP.bf16(w))
    a1 = np.abs(x) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    a2 = a1 @ np.abs(p["W2"]).T + np.abs(p["b2"])
    return a2 @ np.abs(p["W3"]) + abs(p["b3"][0])


def _solver0():
    import paper_2607_06045_amd as P
    return P.Solver(3)


def test_mlp_forward_parity():
    s = _solver0()
    w = MLP.init(1)
    s.mlp_set_weights(w)
    assert np.array_equal(s.mlp_get_weights(), w)
    x = np.random.default_rng(0).uniform(0, 1, (3001, 16)).astype(np.float32)
    y = s.mlp_forward(x)
    ref = MLP.forward(w, x.astype(np.float64))[0]
    tol = 2 * 144 * 2.0 ** -24 * _abs_scale(w, x.astype(np.float64))
    print(f"forward: max |dy| {np.abs(y - ref).max():.2e}, max tol {tol.max():.2e}", flush=True)
    assert (np.abs(y - ref) <= tol).all()
    import torch
    yd = s.mlp_forward(torch.from_numpy(x).cuda())
    assert np.array_equal(yd.cpu().numpy(), y)


def test_mlp_gradient_parity_and_determinism():
    s = _solver0()
    w = MLP.init(2)
    s.mlp_set_weights(w)
    rng = np.random.default_rng(1)
    for B in (1, 63, 64, 1000, 70001):
        x = rng.uniform(0, 1, (B, 16)).astype(np.float32)
        t = rng.uniform(0, 0.5, B).astype(np.float32)
        g, loss = s.mlp_grad(x, t)
        lr_, gr = MLP.loss_and_grad(w, x.astype(np.float64), t.astype(np.float64))
        rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
        print(f"grad B={B}: loss {loss:.6e} vs {lr_:.6e}, rel err {rel:.2e}", flush=True)
        assert rel < 1e-4 and abs(loss - lr_) <= 1e-5 * lr_
        g2, loss2 = s.mlp_grad(x, t)
        assert np.array_equal(g, g2) and loss == loss2


def test_mlp_adam_parity():
    s = _solver0()
    w = MLP.init(3)
    s.mlp_set_weights(w)
    opt = MLP.Adam(w)
    rng = np.random.default_rng(2)
    lr = 1e-3
    for it in range(5):
        x = rng.uniform(0, 1, (512, 16)).astype(np.float32)
        t = rng.uniform(0, 0.5, 512).astype(np.float32)
        lg = s.mlp_train_step(x, t, lr)
        lo = opt.step(x.astype(np.float64), t.astype(np.float64), lr)
        assert abs(lg - lo) <= 1e-4 * lo
    wg = s.mlp_get_weights()
    d = np.abs(wg - opt.w)
    print(f"adam 5 steps: max |dw| {d.max():.2e} (lr {lr}), moved {np.abs(opt.w - w).max():.2e}", flush=True)
    # each step moves a weight by at most about lr; the two sides agree to a
    # small fraction of a step
    assert d.max() <= 0.05 * lr


def test_learned_indicator_trains_on_gpu():
    """Features and Hennemann alpha of synthetic blasts and shear layers are
    the training data; the network learns them on the GPU and then serves as
    DGIDP_IND_MLP."""
    import paper_2607_06045_amd as P
    import torch
    xs, ts = [], []
    for k, (mesh_fn, u_fn) in enumerate([
            (lambda: workload_mesh("blast22k"), lambda x, y: states.sedov_gaussian(x, y, sigma=0.05)),
            (lambda: workload_mesh("blast22k"), lambda x, y: states.sedov_tophat(x, y)),
            (lambda: random_mesh(2, 16, 1, 0.3, L=2.0, x0=-1.0, y0=-1.0),
             lambda x, y: states.shear_layer(x, y, seed=7)),
            (lambda: random_mesh(5, 12, 1, 0.3), lambda x, y: states.quadrants(x, y))]):
        s, u = _solver(mesh_fn(), 3, u_fn)
        for _ in range(3 if k < 2 else 1):
            xs.append(s.features(device=True))
            ts.append(s.indicator(P.IND_HENNEMANN, device=True))
            s.step(0.5)
    X = torch.cat(xs)
    Y = torch.cat(ts)
    print(f"training set: {X.shape[0]} elements, {(Y > 0).float().mean().item():.3f} troubled", flush=True)
    net = P.Solver(3)
    net.mlp_set_weights(MLP.init(11))
    g = torch.Generator(device="cuda").manual_seed(0)
    first = None
    for it in range(600):
        idx = torch.randint(0, X.shape[0], (4096,), device="cuda", generator=g)
        loss = net.mlp_train_step(X[idx], Y[idx], 2e-3)
        first = loss if first is None else first
    full = ((net.mlp_forward(X) - Y) ** 2).mean().item()
    base = ((Y - Y.mean()) ** 2).mean().item()
    print(f"train: first batch loss {first:.3e}, final full-set mse {full:.3e}, "
          f"variance of the target {base:.3e}", flush=True)
    assert full < 0.25 * base
    # the trained network as the context's indicator
    s, u = _solver(workload_mesh("blast22k"), 3, lambda x, y: states.workload_state("blast22k", x, y))
    s.mlp_set_weights(net.mlp_get_weights())
    a = s.indicator(P.IND_MLP)
    assert np.array_equal(a, s.mlp_forward(s.features()))


def test_mlp_errors():
    import paper_2607_06045_amd as P
    s = _solver0()
    with pytest.raises(P.DgidpError):
        s.mlp_forward(np.zeros((4, 16), np.float32))  # no weights yet
    s.mlp_set_weights(MLP.init(0))
    with pytest.raises(ValueError):
        s.mlp_forward(np.zeros((4, 15), np.float32))
    bad = MLP.init(0)
    bad[7] = np.nan
    with pytest.raises(P.DgidpError):
        s.mlp_set_weights(bad)
    with pytest.raises(P.DgidpError):
        s.mlp_train_step(np.zeros((4, 16), np.float32), np.zeros(4, np.float32), 0.0)


def test_learned_indicator_drives_amr():
    """The network trained on GPU-generated (features, modal indicator) pairs
    drives dynamic AMR of the blast: its refine / keep / coarsen decisions agree
    with the modal indicator's on the same states, and the run stays within
    the positivity bounds."""
    from paper_2607_06045_amd import evaluate as EV
    r = EV.run_learned(steps=40, iters=1500, blasts=2, shears=1, snaps=4)
    print({k: r[k] for k in ("agreement", "refine_recall", "coarsen_recall", "violations",
                             "l1_density_base_cells", "indicator_ms")}, flush=True)
    print("elements plain", r["elements"]["plain"], "learned", r["elements"]["learned"], flush=True)
    assert r["agreement"] > 0.9 and r["refine_recall"] > 0.9
    assert r["violations"] == {"plain": 0, "learned": 0}
    assert r["l1_density_base_cells"] < 1e-2 * r["l1_density_scale"]


def test_mixed_precision_amr_run():
    """Shear layer with dynamic AMR (the mixed run replays the FP64 run's
    flags): mixed against FP64 within 1e-5 relative L1 per variable, zero
    violations, and both conserve to round-off across the adaptations."""
    from paper_2607_06045_amd import evaluate as EV
    r = EV.run_mixed(40)
    print(r, flush=True)
    assert max(r["rel_l1_per_variable"]) < 1e-5
    assert r["violations"] == {"fp64": 0, "mixed": 0}
    assert max(r["conservation_defect"]["fp64"]) < 1e-13
    assert max(r["conservation_defect"]["mixed"]) < 1e-9
