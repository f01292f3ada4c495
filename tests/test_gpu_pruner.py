"""GPU parity of the learned window pruner against the FP64 oracle, through
the C ABI: the fused cell map, the network's forward pass, the gradient of
the class-weighted BCE, Adam, and the window labels."""
import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O
from oracle import pruner_oracle as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).to(DEV)


@pytest.mark.parametrize("w,h,seed", [(64, 128, 1), (200, 136, 2), (640, 480, 3), (1242, 375, 4), (503, 260, 5),
                                      (1000, 16, 6)])
def test_cellmap_matches_oracle(w, h, seed):
    img = pd_synth.frame(w, h, seed)
    print(f"\n[cellmap] {w}x{h}", flush=True)
    blocks, cells, cmap = pd.features_cellmap(to_dev(img))
    torch.cuda.synchronize()
    exp = P.cellmap(img).transpose(2, 0, 1)
    got = cmap.cpu().numpy().astype(np.float64)
    assert got.shape == exp.shape
    # LBP channels: counts / 64 are exact
    assert np.array_equal(got[9:], exp[9:])
    err = np.abs(got[:9] - exp[:9])
    assert np.all(err <= 1e-4 * np.abs(exp[:9]) + 2e-6), err.max()
    # the fused pass leaves the features bitwise equal to pd_features
    b2, c2 = pd.features(to_dev(img))
    assert torch.equal(blocks.view(torch.int32), b2.view(torch.int32))
    assert torch.equal(cells, c2)


def _maps(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for hc, wc in sizes:
        m = rng.random((68, hc, wc))
        m[:9] = m[:9] / np.sqrt((m[:9] ** 2).sum(axis=0, keepdims=True))  # HOG-like unit vectors
        out.append(m.astype(np.float32))
    return out


SIZES = [(6, 5), (20, 30), (17, 70), (1, 129)]


def test_forward_matches_oracle():
    params = pd_synth.pruner_init(seed=3)
    params[33505 - 17:33505 - 1] *= 3.0
    maps = _maps(SIZES, 10)
    b = pd.PrunerBatch([to_dev(m) for m in maps])
    logits = b.forward(to_dev(params))
    torch.cuda.synchronize()
    for m, z in zip(maps, logits):
        exp, _ = P.forward(m.transpose(1, 2, 0).astype(np.float64), params.astype(np.float64))
        got = z.cpu().numpy()
        assert np.abs(got - exp).max() <= 1e-5 * max(1.0, np.abs(exp).max()), np.abs(got - exp).max()


def _labels(maps, seed):
    rng = np.random.default_rng(seed)
    labs = [(rng.random(m.shape[1:]) < 0.15).astype(np.float32) for m in maps]
    masks = [(rng.random(m.shape[1:]) < 0.85).astype(np.float32) for m in maps]
    return labs, masks


def test_gradient_matches_oracle_and_is_deterministic():
    params = pd_synth.pruner_init(seed=4)
    maps = _maps(SIZES, 11)
    labs, masks = _labels(maps, 12)
    pw = 6.0
    b = pd.PrunerBatch([to_dev(m) for m in maps], [to_dev(l) for l in labs], [to_dev(k) for k in masks])
    g1 = b.gradient(to_dev(params), pw).clone()
    st = b.stats.clone()
    g2 = b.gradient(to_dev(params), pw).clone()
    torch.cuda.synchronize()
    assert torch.equal(g1.view(torch.int32), g2.view(torch.int32))
    p64 = params.astype(np.float64)
    xs = [m.transpose(1, 2, 0).astype(np.float64) for m in maps]
    zs, caches = zip(*[P.forward(x, p64) for x in xs])
    loss, dz = P.bce_loss_grad(zs, [l.astype(np.float64) for l in labs], [k.astype(np.float64) for k in masks], pw)
    exp = sum(P.backward(d, c, p64) for d, c in zip(dz, caches))
    got = g1.cpu().numpy().astype(np.float64)
    s = st.cpu().numpy()
    assert s[1] == sum(k.sum() for k in masks)
    assert abs(s[0] - loss) <= 1e-6 * abs(loss), (s[0], loss)
    o = 0
    for cin, cout in [(68, 32), (32, 32), (32, 16)]:
        for n in (cout * cin * 9, cout):
            e, gg = exp[o:o + n], got[o:o + n]
            assert np.abs(gg - e).max() <= 1e-5 * np.abs(e).max(), (o, n, np.abs(gg - e).max(), np.abs(e).max())
            o += n
    e, gg = exp[o:], got[o:]
    assert np.abs(gg - e).max() <= 1e-5 * np.abs(e).max()


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    n = 33505
    p, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = (0.1 * rng.normal(size=n)).astype(np.float32), (0.01 * rng.random(n)).astype(np.float32)
    tp, tg, tm, tv = to_dev(p), to_dev(g), to_dev(m), to_dev(v)
    pd.adam_step(tp, tg, tm, tv, 3, lr=1e-3)
    torch.cuda.synchronize()
    # the hyper-parameters cross the C ABI as float32: give the oracle the same values
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    ep, em, ev = P.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                             v.astype(np.float64), 3, lr=f32(1e-3), beta1=f32(0.9), beta2=f32(0.999),
                             eps=f32(1e-8))
    assert np.abs(tm.cpu().numpy() - em).max() <= 1e-6 * np.abs(em).max()
    assert np.abs(tv.cpu().numpy() - ev).max() <= 1e-6 * np.abs(ev).max()
    assert np.abs(tp.cpu().numpy() - ep).max() <= 1e-6 * np.abs(ep).max()


def test_window_labels_match_oracle():
    rng = np.random.default_rng(6)
    hc, wc = 40, 29
    scores = rng.normal(size=(hc - 15, wc - 7)).astype(np.float32)
    thr = to_dev(np.array([0.8]))
    lab, mask = pd.window_labels(to_dev(scores), wc, hc, thr)
    torch.cuda.synchronize()
    el, em = P.window_labels(hc, wc, scores.astype(np.float64), 0.8)
    assert np.array_equal(lab.cpu().numpy(), el) and np.array_equal(mask.cpu().numpy(), em)


@pytest.mark.parametrize("w,h,seed", [(64, 128, 21), (640, 480, 22), (1242, 375, 23), (333, 200, 24)])
def test_bf16_inference_logits_match_oracle(w, h, seed):
    """Cell map (BF16, channels-last) and the network on BF16 MFMA against the
    FP64 oracle: BF16 rounding of the inputs, weights and two layer outputs
    bounds the error at a few 1e-3 of the logit scale."""
    img = pd_synth.frame(w, h, seed)
    params = pd_synth.pruner_init(seed=seed)
    print(f"\n[bf16 logits] {w}x{h}", flush=True)
    got = pd.pruner_logits_bf16(to_dev(img), to_dev(params)).cpu().numpy().astype(np.float64)
    exp, _ = P.forward(P.cellmap(img), params.astype(np.float64))
    scale = np.abs(exp).max()
    err = np.abs(got - exp).max()
    print(f"[bf16 logits] max |err| {err:.3g}, max |z| {scale:.3g}", flush=True)
    assert err <= 2e-2 * scale
