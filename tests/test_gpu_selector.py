"""GPU tests of the learned selection path: MLP kernels against the FP64
oracle, device features against their numpy definition, device argmin
selection, and bit-exact results whatever the selection."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as R
from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from tests import gpu_util
    E = gpu_util.lib()
    return E, torch


def test_mlp_forward_and_gradient_match_fp64(env):
    E, torch = env
    k = 6
    rng = np.random.default_rng(10)
    net = E.MLP(k, seed=3)
    p = net.get_params().astype(np.float64)
    p[-k:] = rng.normal(0, 0.1, k)
    net.set_params(p.astype(np.float32))
    p32 = net.get_params().astype(np.float64)
    for B in (1, 63, 64, 65, 300):
        x = rng.normal(0, 1, (B, 16)).astype(np.float32)
        t = rng.normal(0, 1, (B, k)).astype(np.float32)
        dx = torch.from_numpy(x).cuda()
        dt = torch.from_numpy(t).cuda()
        y = torch.zeros((B, k), dtype=torch.float32, device="cuda")
        net.forward(dx.data_ptr(), B, y.data_ptr())
        g = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        net.grad(dx.data_ptr(), dt.data_ptr(), B, g.data_ptr(), loss.data_ptr())
        torch.cuda.synchronize()
        y_ref, _ = R.forward(p32, x.astype(np.float64), k)
        g_ref = R.grad(p32, x.astype(np.float64), t.astype(np.float64), k)
        l_ref = R.loss(p32, x.astype(np.float64), t.astype(np.float64), k)
        ey = np.max(np.abs(y.cpu().numpy() - y_ref)) / max(1.0, np.max(np.abs(y_ref)))
        gg = g.cpu().numpy().astype(np.float64)
        eg = np.max(np.abs(gg - g_ref)) / max(np.max(np.abs(g_ref)), 1e-12)
        el = abs(float(loss.item()) - l_ref) / max(l_ref, 1e-12)
        _say(f"B={B}: forward rel {ey:.2e}, grad rel {eg:.2e}, loss rel {el:.2e}")
        assert ey <= 1e-5 and eg <= 1e-4 and el <= 1e-5
    net.free()


def test_mlp_training_reduces_loss(env):
    E, torch = env
    k = 4
    rng = np.random.default_rng(11)
    n = 4096
    x = rng.normal(0, 1, (n, 16))
    x[:, -1] = 1.0
    A = rng.normal(0, 0.5, (16, k))
    y = np.tanh(x @ A) + 0.01 * rng.normal(0, 1, (n, k))
    from paper_1402_4466_amd import mlp as M
    model, hist = M.train(x, y, epochs=30, batch=256, lr=3e-3, seed=2)
    assert hist[-1] < 0.2 * hist[0], hist
    # folded weights give the same predictions on raw inputs as the trained net on standardised inputs
    mu, sd = np.asarray(model["mu"]), np.asarray(model["sigma"])
    xs = (x - mu) / sd
    xs[:, -1] = 1.0
    y_std, _ = R.forward(np.asarray(model["params_raw"]), xs, k)
    y_fold, _ = R.forward(np.asarray(model["params_folded"]), x, k)
    assert np.allclose(y_std, y_fold, rtol=1e-4, atol=1e-4)


def test_device_features_match_definition(env):
    E, torch = env
    from paper_1402_4466_amd import selector as S
    n_bits = 3 * 65536 + 100
    pool_n = 50
    d = D.pool_densities(pool_n, seed=31)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(31, i) for i in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    qs = D.queries(32, 80, pool_n, 2, 40)
    feat = torch.zeros((len(qs), 16), dtype=torch.float32, device="cuda")
    E.query_features(bms, [(q.idx, q.T) for q in qs], feat.data_ptr())
    got = feat.cpu().numpy().astype(np.float64)
    want = S.features_host([(q.idx, q.T) for q in qs], [b.stats() for b in bms], n_bits)
    assert np.allclose(got, want, rtol=2e-4, atol=2e-4), np.max(np.abs(got - want))
    for b in bms:
        b.release()


def test_learned_selection_keeps_results_bit_exact(env):
    E, torch = env
    from paper_1402_4466_amd import mlp as M
    from paper_1402_4466_amd import selector as S
    from tests import gpu_util as G
    n_bits = 2 * 65536 + 77
    pool_n = 60
    d = D.pool_densities(pool_n, seed=41)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(41, i) for i in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    qs = D.queries(42, 30, pool_n, 2, 30)
    outs = [G.alloc_out(n_bits, int(sum(len(pool[i]) for i in q.idx))) for q in qs]
    batch = E.Batch(bms, [(q.idx, q.T) for q in qs], [o[0].data_ptr() for o in outs], [o[2] for o in outs],
                    [o[1].data_ptr() for o in outs])
    codes = S.arm_codes()
    # an untrained (random) network: any selection must give identical outputs
    rng = np.random.default_rng(5)
    model = {"kind": "mlp", "n_out": len(codes), "arm_codes": codes,
             "params_folded": rng.normal(0, 0.3, M.NI * M.H + M.H + M.H * M.H + M.H + M.H * len(codes) + len(codes)).tolist()}
    sel = S.MLPSelector(model)
    sel.apply(batch, bms, qs, n_bits)
    chosen = batch.get_variants()
    assert set(chosen.tolist()) <= set(codes)
    # argmin agrees with the predictions
    feat = torch.zeros((len(qs), 16), dtype=torch.float32, device="cuda")
    batch.features(feat.data_ptr())
    arms = sel.choose_device_arms(feat.data_ptr(), len(qs))
    assert [codes[a] for a in arms] == chosen.tolist()
    batch.run()
    torch.cuda.synchronize()
    for i, q in enumerate(qs):
        want, _ = O.threshold([pool[j] for j in q.idx], n_bits, q.T, want_hist=False)
        assert np.array_equal(G.fetch(outs[i][0], outs[i][1]), want)
    assert E.device_errors() == 0
    batch.free()
    sel.predictor().free()
    for b in bms:
        b.release()
