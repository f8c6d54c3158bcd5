"""CPU tests of the library boundary and the host-side logic around it.

* the built library loads and exports every function the public header declares;
* the pure host entry points (output bound, variant codes) follow their documented
  definitions; the bound is checked against true canonical output sizes computed by
  the oracle;
* selector host logic: the feature definition, the library's model-file reader and
  writer, and its exact folding of input standardisation into the first MLP layer
  (the rule-set fit is checked on the GPU, since training runs there).

No GPU work is started here.
"""
import os
import re

import numpy as np
import pytest

from oracle import mlp_ref as R
from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ewahthr.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    names = set(re.findall(r"\b(ewah_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def E():
    from paper_1402_4466_amd import ewahthr
    return ewahthr


def test_library_exports_every_declared_function(E):
    import ctypes
    lib = ctypes.CDLL(E.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 30, declared
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(E.EXPORTED) == declared


def test_output_bound_definition_and_true_sizes(E):
    assert E.output_bound(0, 10) == 0
    assert E.output_bound(64, 1) == 2
    assert E.output_bound(64 * 100, 10**9) == 101
    assert E.output_bound(64 * 100, 3) == 4
    rng = np.random.default_rng(7)
    for case in range(40):
        n_bits = int(rng.integers(1, 5000))
        n = int(rng.integers(1, 7))
        dens = np.clip(rng.uniform(0.0, 1.0, n) ** 3, 1e-3, 0.999)
        keys = [D.key(900 + case, i) for i in range(n)]
        if case % 2:
            streams = D.bitmaps(D.MARKOV, 8.0, 8.0 * (1.0 - dens) / dens, n_bits, keys)
        else:
            streams = D.bitmaps(D.IID, dens, 0.0, n_bits, keys)
        total = sum(len(s) for s in streams)
        bound = E.output_bound(n_bits, total)
        for T in range(0, n + 2):
            out, _ = O.threshold(streams, n_bits, T, want_hist=False)
            assert len(out) <= bound, (case, T, len(out), bound)


def test_variant_codes(E):
    d = E.default_variant()
    assert d == E.variant_code(True, 8, 8)
    c = E.variant_code(False, 64, 200)
    assert c & 1 == 0 and (c >> 8) & 0xFF == 64 and (c >> 16) & 0xFF == 200
    assert E.variant_code(True, 0, 0) & 1 == 1
    lp = E.variant_code(False, 8, 8, looped=True)
    assert lp == E.variant_code(False, 8, 8) | (1 << 24) and not E.variant_code(False, 8, 8) & (1 << 24)
    from paper_1402_4466_amd import selector as S
    codes = S.arm_codes()
    assert len(set(codes)) == len(codes) == len(S.ARMS)


def test_features_definition_on_known_stats():
    from paper_1402_4466_amd import selector as S
    n_bits = 1 << 20
    stats = [dict(n_words=100, n_literals=60, popcount=1 << 10, run_count=40),
             dict(n_words=300, n_literals=200, popcount=1 << 14, run_count=90),
             dict(n_words=7, n_literals=0, popcount=0, run_count=0)]
    f = S.features_host([([0, 1], 2), ([1, 2, 0], 1)], stats, n_bits)
    assert f.shape == (2, S.N_FEATURES)
    q0 = f[0]
    assert q0[0] == 1.0 and q0[1] == 1.0 and q0[2] == 1.0 and q0[3] == 0.0   # log2 N, log2 T, T/N, log2(N-T+1)
    assert np.isclose(q0[4], (-10 + -6) / 2) and q0[5] == -6 and q0[6] == -10
    assert np.isclose(q0[7], 2.0)
    assert np.isclose(q0[8], np.log2(131)) and np.isclose(q0[9], np.log2(91))
    assert np.isclose(q0[10], np.log2(401)) and np.isclose(q0[11], np.log2(301))
    assert np.isclose(q0[12], 260 / 400) and q0[13] == 20 and q0[15] == 1.0
    assert np.isclose(q0[14], (2**-10 + 2**-6) / 2)
    # an empty bitmap's density is floored, not log(0)
    assert np.isfinite(f[1]).all() and np.isclose(f[1][6], np.log2(1e-9))


def test_standardisation_fold_is_exact(E):
    """The library folds the features' standardisation into the first layer
    (W1' = W1 / sigma, b1' = b1 - (mu / sigma) W1) when a model file has no folded
    parameters; the saved folded network on raw features equals the raw network on
    standardised features (FP64 reference forward)."""
    import json
    import tempfile
    rng = np.random.default_rng(4)
    k = 5
    n_par = int(E._mlp_num_params(k))
    p = rng.normal(0, 0.3, n_par)
    mu = rng.normal(3.0, 2.0, 16)
    sd = rng.uniform(0.5, 3.0, 16)
    mu[-1], sd[-1] = 0.0, 1.0
    coef = rng.uniform(0.0, 1.0, (5, k))
    with tempfile.TemporaryDirectory() as d:
        src, dst = os.path.join(d, "m.json"), os.path.join(d, "m2.json")
        with open(src, "w") as f:
            json.dump({"kind": "mlp", "n_out": k, "arm_codes": [11, 22, 33, 44, 55], "mu": mu.tolist(),
                       "sigma": sd.tolist(), "params_raw": p.tolist(), "rules_coef": coef.tolist(),
                       "eval": {"ignored": [1, {"s": "x\u00e9"}]}}, f)
        sel = E.Selector.load(src)
        assert sel.n_arms == k and sel.arm_codes().tolist() == [11, 22, 33, 44, 55]
        sel.save(dst)
        sel.free()
        with open(dst) as f:
            m2 = json.load(f)
    X = rng.normal(3.0, 2.0, (200, 16))
    X[:, -1] = 1.0
    Xs = (X - mu) / sd
    y_std, _ = R.forward(np.asarray(m2["params_raw"]), Xs, k)
    y_fold, _ = R.forward(np.asarray(m2["params_folded"]), X, k)
    assert np.allclose(y_std, y_fold, rtol=1e-5, atol=1e-5)
    assert np.allclose(np.asarray(m2["rules_coef"]).ravel(), coef.ravel())


def test_selector_model_errors(E):
    import json
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        bad = os.path.join(d, "bad.json")
        for body in ('{"kind": "mlp", "arm_codes": [1, 2]', '{"kind": "mlp", "arm_codes": [1, 2], "mu": [0]}',
                     '[1, 2, 3]'):
            with open(bad, "w") as f:
                f.write(body)
            with pytest.raises(E.EwahError) as e:
                E.Selector.load(bad)
            assert e.value.code == E.EFORMAT, body
        with pytest.raises(E.EwahError) as e:
            E.Selector.load(os.path.join(d, "missing.json"))
        assert e.value.code == E.EINVAL
        ok = os.path.join(d, "ok.json")
        with open(ok, "w") as f:
            json.dump({"arm_codes": [7], "mu": [0.0] * 16, "sigma": [1.0] * 16,
                       "params_raw": [0.0] * int(E._mlp_num_params(1))}, f)
        sel = E.Selector.load(ok)
        assert sel.n_arms == 1
        sel.free()
