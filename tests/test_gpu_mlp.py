"""The learned (k, p, q) predictor on the device against the FP64 oracle:
He init, forward, gradients (P13: FP32 kernels vs the analytic FP64 gradient,
1e-4 relative), Adam steps, a short training run, the pilot features, and the
end-to-end learned sizing with its a-posteriori check and adaptive fallback."""

import math

import numpy as np
import pytest

import synth
from oracle import mlp as omlp

from gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _f32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


def _theta64(net):
    return net.params.cpu().numpy().astype(np.float64)


def test_init_matches_oracle():
    import paper_2307_15572_amd as rs
    announce("mlp init")
    net = rs.Mlp(seed=21)
    got = _theta64(net)
    ref = omlp.he_init(21)
    # the same Philox / Box-Muller draws, rounded to FP32 (transcendentals may
    # differ by an ulp of FP64 between the device and the host library)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref) + 1e-12)


def test_forward_hand_computed():
    # the hand-worked parameters and outputs of the oracle pin: every value
    # in them is exact in FP32
    import paper_2307_15572_amd as rs
    from test_oracle_mlp import HAND_X, HAND_Y, _hand_params
    announce("mlp forward, hand-computed parameters")
    net = rs.Mlp(seed=0)
    net.params.copy_(_f32(_hand_params()))
    y = net.forward(_f32(HAND_X)).cpu().numpy().astype(np.float64)
    assert np.allclose(y, HAND_Y, rtol=0, atol=1e-6)


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-3.0, 0.0, size=(B, 16))
    T = rng.standard_normal((B, 3))
    return X, T


@pytest.mark.parametrize("B", [1, 37, 128])
def test_forward_and_gradient_match_oracle(B):
    import paper_2307_15572_amd as rs
    announce(f"mlp forward / grad B={B}")
    net = rs.Mlp(seed=5)
    X, T = _batch(B, B)
    X = X.astype(np.float32).astype(np.float64)
    T = T.astype(np.float32).astype(np.float64)
    theta = _theta64(net)
    y_ref, _ = omlp.forward(theta, X)
    y = net.forward(_f32(X)).cpu().numpy()
    assert np.abs(y - y_ref).max() <= 1e-5 * max(1.0, np.abs(y_ref).max())
    L, g = net.grad(_f32(X), _f32(T))
    L_ref, g_ref = omlp.grad(theta, X, T)
    assert abs(L - L_ref) <= 1e-5 * L_ref
    g = g.cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()


def test_forward_large_batch_spans_workgroups():
    import paper_2307_15572_amd as rs
    announce("mlp forward B=1000")
    net = rs.Mlp(seed=6)
    X, _ = _batch(1000, 3)
    y = net.forward(_f32(X)).cpu().numpy()
    y_ref, _ = omlp.forward(_theta64(net), X.astype(np.float32).astype(np.float64))
    assert np.abs(y - y_ref).max() <= 1e-5 * max(1.0, np.abs(y_ref).max())


def test_adam_steps_track_oracle():
    import paper_2307_15572_amd as rs
    announce("mlp adam steps")
    net = rs.Mlp(seed=8)
    X, T = _batch(96, 4)
    X = X.astype(np.float32).astype(np.float64)
    T = T.astype(np.float32).astype(np.float64)
    theta = _theta64(net)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    gmin = np.full_like(theta, np.inf)
    for t in range(1, 6):
        _, g = omlp.grad(theta, X, T)
        gmin = np.minimum(gmin, np.abs(g) / np.abs(g).max())
        theta, m, v = omlp.adam_step(theta, m, v, g, t, lr=1e-3)
        net.train_step(_f32(X), _f32(T), lr=1e-3)
    got = _theta64(net)
    # Adam divides each gradient by its own magnitude: where the FP64 gradient
    # is well above the FP32 kernels' error at every step the updates agree to
    # FP32 rounding; elsewhere each of the 5 steps moves a weight by <= lr
    sure = gmin >= 1e-2
    assert sure.sum() > 1000
    assert np.abs(got - theta)[sure].max() <= 5e-6
    assert np.abs(got - theta).max() <= 2 * 5 * 1e-3 + 1e-6


def test_training_reduces_loss_like_oracle():
    import paper_2307_15572_amd as rs
    announce("mlp training 40 epochs")
    rng = np.random.default_rng(9)
    X = rng.uniform(-3.0, 0.0, size=(384, 16)).astype(np.float32).astype(np.float64)
    W = rng.standard_normal((3, 16)) / 4
    T = (X @ W.T).astype(np.float32).astype(np.float64)
    net = rs.Mlp(seed=9)
    theta0 = _theta64(net)
    L0 = omlp.loss(theta0, X, T)
    theta_ref, hist_ref = omlp.train(theta0, X, T, epochs=40, batch=128, lr=3e-3)
    Xd, Td = _f32(X), _f32(T)
    losses = []
    for _ in range(40):
        for b0 in range(0, 384, 128):
            losses.append(net.train_step(Xd[b0:b0 + 128], Td[b0:b0 + 128], lr=3e-3))
    L_gpu = omlp.loss(_theta64(net), X, T)
    L_ref = omlp.loss(theta_ref, X, T)
    assert L_gpu < 0.1 * L0 and L_ref < 0.1 * L0
    assert abs(L_gpu - L_ref) <= 0.25 * L_ref + 1e-4 * L0
    assert abs(float(losses[0].item()) - hist_ref[0]) <= 1e-5 * hist_ref[0]


@pytest.mark.parametrize("n,d", [(400, 12.0), (900, 55.0), (260, 80.0)])
def test_pilot_features_match_oracle(n, d):
    import paper_2307_15572_amd as rs
    announce(f"pilot features n={n} d={d}")
    A, _ = synth.channel(3, n, d, tag=910)
    f, _ = rs.pilot_features(to_dev(A), seed=77, channel=3)
    f = f.cpu().numpy().astype(np.float64)
    ref = omlp.pilot_features(A, seed=77, channel=3)
    # exp(-i/d) spectra: every feature is above -1, far from FP32 noise
    assert ref.min() > -1.0
    assert np.abs(f - ref).max() <= 1e-3


def test_targets_match_oracle():
    import paper_2307_15572_amd as rs
    announce("mlp targets (standardization)")
    rng = np.random.default_rng(31)
    labels = np.stack([rng.integers(5, 3000, 700), rng.choice([8, 16, 32, 64, 128, 192], 700),
                       rng.integers(0, 5, 700)], axis=1)
    net = rs.Mlp(seed=1)
    T = net.targets(labels).cpu().numpy().astype(np.float64)
    Tr, mean, sd = omlp.targets(labels)
    st = net.stats.cpu().numpy().astype(np.float64)
    assert np.allclose(st[:3], mean, rtol=1e-6) and np.allclose(st[3:], sd, rtol=1e-6)
    assert np.abs(T - Tr).max() <= 1e-5


def test_predict_matches_oracle_decode():
    # the decode step on both sides takes the device's FP32 network outputs
    import paper_2307_15572_amd as rs
    announce("mlp predict (forward + sizing rules)")
    rng = np.random.default_rng(32)
    net = rs.Mlp(seed=5)
    net.targets(np.stack([rng.integers(20, 1500, 300), rng.choice([8, 32, 128, 192], 300),
                          rng.integers(0, 5, 300)], axis=1))
    X = rng.uniform(-6.0, 0.0, size=(300, 16))
    n_cap = rng.integers(100, 5000, 300)
    got = net.predict(_f32(X), n_cap)
    y = net.forward(_f32(X)).cpu().numpy().astype(np.float64)
    st = net.stats.cpu().numpy().astype(np.float64)
    want = [omlp.decode(y[b], st[:3], st[3:], int(n_cap[b])) for b in range(300)]
    assert got == want


def test_size_label_matches_oracle():
    import paper_2307_15572_amd as rs
    announce("size label from computed spectra")
    rng = np.random.default_rng(33)
    for t in range(40):
        n = int(rng.integers(300, 6000))
        d = float(rng.uniform(5.0, 90.0))
        count = int(rng.integers(50, 600))
        s = np.exp(-np.arange(count) / d - 0.01 * rng.random(count).cumsum())
        k = int(rng.integers(1, count))
        l_min = int(rng.integers(0, count + 100))
        got = rs.size_label(to_dev(s), k, n, l_min)
        assert got == omlp.size_label(s, k, n, l_min), (t, n, d, count, k, l_min)


def test_save_load_roundtrip(tmp_path):
    import paper_2307_15572_amd as rs
    announce("mlp save / load")
    net = rs.Mlp(seed=8)
    net.targets(np.array([[10, 8, 0], [300, 64, 2], [90, 16, 1]]))
    path = str(tmp_path / "net.bin")
    net.save(path)
    other = rs.Mlp(seed=9)
    other.load(path)
    assert bool((other.params == net.params).all()) and bool((other.stats == net.stats).all())
    bad = tmp_path / "bad.bin"
    bad.write_bytes(open(path, "rb").read()[:-4])
    with pytest.raises(rs.RsvdError):
        other.load(str(bad))


def test_posterior_judge_matches_oracle():
    import paper_2307_15572_amd as rs
    from oracle.adaptive import posterior_judge
    from oracle.method import rsvd as oracle_rsvd
    announce("a-posteriori judge of fixed-l threshold runs")
    m, n = 1000, 800
    A = synth.general(m, n, synth.spectrum_exp(n, 30.0), tag=134)
    for k, p, q, tau in ((60, 20, 1, 1e-2), (230, 60, 2, 1e-3), (100, 8, 0, 1e-6)):
        ref = oracle_rsvd(A, k, p, q, seed=4, rank_mode="rel_threshold", rank_param=tau)
        est, flags = posterior_judge(A, ref.Q, ref.s_all, ref.rank, q, tau, 16, seed=4)
        out = rs.run(to_dev(A), k, p, q, seed=4, rank_mode="rel_threshold", rank_param=tau,
                     posterior=16)
        assert out.rank == ref.rank
        assert abs(out.err_est - est) <= 1e-8 * est + 1e-13, (out.err_est, est)
        judged = rs.FLAG_POSTERIOR_FAIL | rs.FLAG_UNCONVERGED
        assert out.flags & judged == flags, (k, p, q, out.flags, flags)


def _timed(fn):
    import time
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def test_learned_sizing_beats_adaptive_only():
    # train on channels labelled by the method itself (the adaptive FP64
    # finder's rank and spectrum), evaluate on others: every evaluated channel
    # ends with its exact threshold rank and accurate kept values, with fewer
    # streams of A than the adaptive finder alone, and, run as one batch
    # (which the sizes known up front allow), in less wall time
    import paper_2307_15572_amd as rs
    from paper_2307_15572_amd import learned
    announce("learned sizing: 240 train channels (n ~ logU[1500, 4000]) / 60 eval (n ~ logU[600, 2500])")
    tau, seed = 1e-6, 5
    dims, dec = synth.channel_dims(300, 600, 2500, tag=77)
    # training channels large enough that no label's l = k + p reaches n (the
    # features see the spectrum, not the size); evaluation keeps small ones
    tdims, _ = synth.channel_dims(300, 1500, 4000, tag=78)
    dims[:240] = tdims[:240]
    feats, labels, evals = [], [], []
    work = None
    for c, (n, d) in enumerate(zip(dims, dec)):
        n, d = int(n), float(d)
        A, _ = synth.channel_device_rng(c, n, d, tag=77)
        if c >= 240:
            evals.append((c, n, d, A))
            continue
        lab, _ = learned.label_channel(A, tau, seed, c, symmetric=True)
        if lab is None:
            continue
        f, work = rs.pilot_features(A, seed=seed, channel=c, work=work)
        feats.append(f.cpu().numpy())
        labels.append(lab)
        del A
    print(f"[learned] {len(labels)} of 240 training channels labelled")
    assert len(labels) >= 120
    net, loss = learned.train_predictor(np.array(feats), labels, epochs=300)
    assert loss < 0.6
    passes_l = passes_a = fell = 0
    t_l = t_a = 0.0
    truth = {}
    for c, n, d, A in evals:
        k_true = min(n, 1 + int(np.floor(d * np.log(1.0 / tau))))
        sig = synth.spectrum_exp(n, d)
        truth[c] = (k_true, sig)
        (out, work), dt = _timed(lambda: learned.decompose(A, net, tau, seed=seed, channel=c,
                                                            symmetric=True, pilot_work=work))
        t_l += dt
        if out.fell_back:
            print(f"[learned] channel {c} n={n} d={d:.1f} predicted {out.predicted}: {out.reason}")
        assert out.rank == k_true, (c, n, d, out.predicted, out.reason)
        s = out.S.cpu().numpy()
        assert np.max(np.abs(s - sig[: out.rank]) / sig[: out.rank]) <= 1e-6
        passes_l += out.passes
        fell += int(out.fell_back)
        ad, dt = _timed(lambda: learned.run_adaptive(A, tau, seed, c, symmetric=True))
        t_a += dt
        assert ad.rank == k_true
        passes_a += learned.adaptive_passes(ad.blocks, 1, ad.l, n)
    # the same channels as one batch: the sizes are known up front
    outs, t_b = _timed(lambda: learned.decompose_batch([e[3] for e in evals], net, tau, seed,
                                                       [e[0] for e in evals], symmetric=True))
    passes_b = 0
    for (c, n, d, A), out in zip(evals, outs):
        k_true, sig = truth[c]
        assert out.rank == k_true, (c, n, d, out.predicted, out.reason)
        s = out.S.cpu().numpy()
        assert np.max(np.abs(s - sig[: out.rank]) / sig[: out.rank]) <= 1e-6
        passes_b += out.passes
    print(f"[learned] passes {passes_l} (batched {passes_b}) vs adaptive {passes_a}; time "
          f"{t_l:.3f} s one by one, {t_b:.3f} s batched, adaptive {t_a:.3f} s; "
          f"fallbacks {fell}/{len(evals)}")
    assert passes_l < passes_a and passes_b < passes_a
    assert fell <= len(evals) // 3
    assert t_b < t_a
