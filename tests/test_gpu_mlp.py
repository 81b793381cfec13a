"""GPU cost-model MLP kernels against the fp64 oracle: forward pass, loss and
gradient of one batch, the Adam update, a short training trajectory; and the
training / selection entry points on a synthetic tuning database."""
import os

import numpy as np
import pytest
import torch

import paper_1510_06585_amd as sk
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def maxerr(a, b):
    """Largest element-wise |a - b| over the block's largest |b|: a few wrong
    elements in a large block fail this even where the norm-wise check passes."""
    b = np.asarray(b, np.float64)
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


def batch(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 24)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    theta = synth.mlp_init(seed).astype(np.float32)
    theta[1536:1600] = rng.uniform(-0.2, 0.2, 64).astype(np.float32)
    theta[5696:5760] = rng.uniform(-0.2, 0.2, 64).astype(np.float32)
    return X, t, theta


@pytest.mark.parametrize("n", [1, 7, 256, 1000])
def test_forward_matches_oracle(n):
    X, t, theta = batch(n, n)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    sk.mlp_forward(dev(theta), dev(X), y)
    torch.cuda.synchronize()
    ref, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64))
    got = y.cpu().numpy()
    assert relerr(got, ref) <= 1e-5
    # element-wise: every output within 2e-5 of the largest |output| (fp32
    # dot products of <= 64 terms of mixed sign)
    assert maxerr(got, ref) <= 2e-5


@pytest.mark.parametrize("n", [1, 33, 256])
def test_gradient_matches_oracle(n):
    X, t, theta = batch(100 + n, n)
    g = torch.empty(5825, dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    sk.mlp_grad(dev(theta), dev(X), dev(t), g, L)
    torch.cuda.synchronize()
    Lr, gr = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    lerr = abs(float(L.cpu()[0]) - Lr) / abs(Lr)
    assert lerr <= 1e-5
    gg = g.cpu().numpy()
    blocks = ((0, 1536), (1536, 1600), (1600, 5696), (5696, 5760), (5760, 5824), (5824, 5825))
    for lo, hi in blocks:
        assert relerr(gg[lo:hi], gr[lo:hi]) <= 1e-4, (lo, hi)
        assert maxerr(gg[lo:hi], gr[lo:hi]) <= 2e-4, (lo, hi)
    print(f"gradient, {n} samples: loss {lerr:.2e}; worst block norm-wise "
          f"{max(relerr(gg[lo:hi], gr[lo:hi]) for lo, hi in blocks):.2e}, element-wise "
          f"{max(maxerr(gg[lo:hi], gr[lo:hi]) for lo, hi in blocks):.2e}")


def test_adam_step_elementwise():
    """One Adam step from the same fp32 gradient, at steps 1, 2 and 50: every
    first and second moment within 1e-6 of the block's largest value, and
    every parameter's update within 1e-5 of its magnitude bound (the update
    computed from |m0| and |g|) plus one fp32 rounding of the parameter.
    (The kernel's constants are fp32: 1 - 0.999f differs from 0.001 by
    1.3e-5 relative, which reaches the update through the second moment's
    bias correction under a square root, about 6.5e-6.)"""
    rng = np.random.default_rng(31)
    theta = synth.mlp_init(31).astype(np.float32)
    g = rng.normal(scale=1e-2, size=5825).astype(np.float32)
    g[::97] = 0.0                       # exactly-zero gradients: moments stay, update 0
    m0 = rng.normal(scale=1e-3, size=5825).astype(np.float32)
    v0 = np.abs(rng.normal(scale=1e-5, size=5825)).astype(np.float32)
    for step in (1, 2, 50):
        P, M, V = dev(theta), dev(m0), dev(v0)
        sk.mlp_adam(P, dev(g), M, V, step)
        torch.cuda.synchronize()
        th, mo, vo = mlp.adam_step(theta.astype(np.float64), g.astype(np.float64), m0.astype(np.float64),
                                   v0.astype(np.float64), step)
        assert maxerr(M.cpu().numpy(), mo) <= 1e-6, step
        assert maxerr(V.cpu().numpy(), vo) <= 1e-6, step
        upd = P.cpu().numpy().astype(np.float64) - theta
        ref_upd = th - theta.astype(np.float64)
        # the update itself (lr-sized), not just the parameters, element by
        # element.  The first moment beta1 m0 + (1 - beta1) g is an fp32 sum
        # of two terms; where they cancel (zero-initialised biases with a
        # small update) its rounding error is relative to the sum of their
        # magnitudes, not to the result, so the update's 1e-5 is taken
        # relative to the same expression with |m0| and |g|.
        vhat = vo / (1.0 - 0.999 ** step)
        u_abs = 1e-3 * (0.9 * np.abs(m0.astype(np.float64)) + 0.1 * np.abs(g.astype(np.float64))) \
            / (1.0 - 0.9 ** step) / (np.sqrt(vhat) + 1e-8)
        bound = 1e-5 * u_abs + 2.0 ** -23 * np.abs(theta.astype(np.float64))
        assert (np.abs(upd - ref_upd) <= bound).all(), step
        assert (upd[::97] == 0).all() == (ref_upd[::97] == 0).all()


def test_adam_matches_oracle_and_training_trajectory():
    X, t, theta = batch(7, 512)
    P = dev(theta)
    m = torch.zeros(5825, device="cuda")
    v = torch.zeros(5825, device="cuda")
    g = torch.empty(5825, device="cuda")
    L = torch.empty(1, device="cuda")
    th = theta.astype(np.float64)
    mo = np.zeros(5825)
    vo = np.zeros(5825)
    losses = []
    for step in range(1, 41):
        sl = slice(((step - 1) % 4) * 128, ((step - 1) % 4) * 128 + 128)
        sk.mlp_grad(P, dev(X[sl]), dev(t[sl]), g, L)
        sk.mlp_adam(P, g, m, v, step)
        Lr, gr = mlp.loss_and_grad(th, X[sl].astype(np.float64), t[sl].astype(np.float64))
        th, mo, vo = mlp.adam_step(th, gr, mo, vo, step)
        torch.cuda.synchronize()
        losses.append((float(L.cpu()[0]), Lr))
    # same trajectory within fp32 rounding: norm-wise, and element-wise for
    # 99.9% of the parameters (an element whose gradient is rounding noise
    # can take a different Adam direction, so the tail is bounded by the
    # per-step size lr * 1/(1 - beta1) over the 40 steps instead)
    Pg = P.cpu().numpy()
    assert relerr(Pg, th) <= 1e-4
    d = np.abs(Pg.astype(np.float64) - th)
    assert np.quantile(d, 0.999) <= 1e-4 * np.abs(th).max()
    assert d.max() <= 40 * 1e-3 * 10
    assert losses[-1][1] < losses[0][1]
    assert abs(losses[-1][0] - losses[-1][1]) <= 1e-3 * losses[-1][1]


def _masks(comp):
    """Every valid fusion partition of a composition (split bits after each stage
    and, with a reduce, one bit for a separate reduce kernel)."""
    k = len(comp["stages"])
    nbits = k - 1 + (1 if comp["reduce"] else 0)
    out = []
    for m in range(1 << nbits):
        nblur, ok = 0, True
        for i, (n, _) in enumerate(comp["stages"]):
            nblur += n == "blur5"
            ok &= nblur <= 1
            if i < k - 1 and (m >> i) & 1:
                nblur = 0
        if ok:
            out.append(m)
    return out


def _synthetic_db(path, rng):
    """Rows shaped like the tuner's, with runtimes from a known law
    t = bytes / BW + launches * 4 us (+3 us for 64-thread work-groups), over the
    same configuration space the selector scores."""
    rows = 0
    with open(path, "w") as f:
        for c in range(60):
            comp = synth.composition(rng, log2_lo=12, log2_hi=22)
            if comp["domain"] != "u8":
                continue
            root = sk.image_chain(comp["stages"], comp["reduce"])
            proto = [sk.proto([comp["H"], comp["W"], 4], sk.U8)] * 2
            if comp["reduce"] == "hist_sum":
                proto += [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]
            elif comp["reduce"] == "sum":
                proto += [sk.proto([4], sk.U64)]
            for m in _masks(comp):
                for wg in (64, 256):
                    o = {"fusion": sk.FUSE_MASK, "split_mask": m, "wg": wg}
                    feat = sk.features(root, proto, o)
                    t_us = 2.0 ** feat[22] / 5e6 + 4.0 * 2.0 ** feat[23] + (3.0 if wg == 64 else 0.0)
                    f.write(f"c{c},{sk.FUSE_MASK},{m},0,{wg},1,0," + ",".join(f"{x:.6g}" for x in feat)
                            + f",{t_us:.4f},{t_us:.4f}\n")
                    rows += 1
    return rows


def test_cost_train_and_select_on_synthetic_law(tmp_path):
    rng = np.random.default_rng(11)
    db = str(tmp_path / "db.csv")
    assert _synthetic_db(db, rng) > 100
    w0 = str(tmp_path / "w0.txt")
    w = str(tmp_path / "w.txt")
    l0 = sk.cost_train(db, w0, 0, seed=3)
    l1 = sk.cost_train(db, w, 300, seed=3)
    assert l1 < 0.1 * l0
    # the trained model prefers the fused plan of an unseen chain
    comp_root = sk.image_chain([("noise", {"seed": 1}), ("solarise", {}), ("mirror", {})], "hist_sum")
    proto = [sk.proto([1024, 1024, 4], sk.U8)] * 2 + [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]
    o = sk.cost_select(comp_root, proto, w)
    d = sk.Plan(comp_root, proto, o).describe()
    assert len(d["kernels"]) == 1
    assert os.path.getsize(w) > 1000
    # the ranked shortlist: best first, distinct, increasing predicted time,
    # led by cost_select's choice, and capped by the number of valid configs
    ranked = sk.cost_rank(comp_root, proto, w, 6)
    assert len(ranked) == 6 and ranked[0][0] == o
    preds = [p for _, p in ranked]
    assert all(a <= b for a, b in zip(preds, preds[1:])) and preds[0] > 0
    keys = {tuple(sorted(r.items())) for r, _ in ranked}
    assert len(keys) == 6
    n_valid = sk.config_count(comp_root, proto)
    everything = sk.cost_rank(comp_root, proto, w, n_valid + 10)
    assert len(everything) == n_valid
    with pytest.raises(sk.SkelError):
        sk.cost_rank(comp_root, proto, w, 0)


def test_trained_model_against_the_methods_without_it(tmp_path):
    """A scaled-down selector experiment (400 training compositions x 16
    sampled configurations, 40 held-out compositions timed exhaustively, the
    default plan and the re-timings measured with the tuner's own protocol):
    the network trained on the GPU picks plans within 10% of the exhaustive
    best on mean (the target), far better than the untrained network and a
    random configuration, and the labels it is scored against repeat within 3%
    (median) when each held-out composition's best and runner-up are re-timed.
    The default plan and the paper's nearest-neighbour derivation are
    reported, not asserted: at this scale their order against the model
    varies (full-size results are in the benchmark's selector extra)."""
    from paper_1510_06585_amd import selector
    r = selector.experiment(n_train=400, n_test=40, per_train=16, seed=7, epochs=200, workdir=str(tmp_path),
                            log=lambda *a: None)
    reg = r["regret"]
    print({k: v["mean"] for k, v in reg.items()}, r["label_noise"]["rel_diff"])
    assert reg["model"]["mean"] <= 0.10
    assert reg["model_ensemble3"]["mean"] <= 0.10
    assert reg["model"]["mean"] < 0.5 * reg["untrained"]["mean"]
    assert reg["model"]["mean"] < 0.5 * reg["random"]["mean"]
    assert r["label_noise"]["rel_diff"]["median"] < 0.03
