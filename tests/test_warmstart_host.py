"""Host-side checks of the warm-start network definition: the weight-blob
layout matches include/pot.h, the features reproduce the cost, and the
reference forward has the symmetries the design relies on."""
import os
import re

import numpy as np

from paper_2601_17196_amd import instances as I
from paper_2601_17196_amd import warmstart as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _random_weights(seed=0, scale=0.3):
    g = np.random.default_rng(seed)
    H = W.HID
    return {"W1": g.normal(0, scale, (H, W.NFEAT)), "b1": g.normal(0, 0.1, H),
            "W2": g.normal(0, scale / np.sqrt(H) * 3, (H, H)), "b2": g.normal(0, 0.1, H),
            "W3a": g.normal(0, scale / np.sqrt(H) * 3, (H, H)), "W3b": g.normal(0, scale / np.sqrt(H) * 3, (H, H)),
            "b3": g.normal(0, 0.1, H), "w4": g.normal(0, 0.1, H), "b4": np.array([0.05])}


def test_blob_layout_matches_header():
    src = open(os.path.join(ROOT, "include", "pot.h")).read()
    assert int(re.search(r"#define POT_WARM_WEIGHT_BYTES (\d+)", src).group(1)) == W.BLOB_BYTES
    arr = _random_weights()
    blob = W.pack_blob(arr)
    fp = blob[:W.BF16_OFFSET].view(np.float32)
    assert np.array_equal(fp[W.F_B2:W.F_B2 + W.HID], arr["b2"].astype(np.float32))
    assert fp[W.F_B4] == np.float32(arr["b4"][0])
    bf = blob[W.BF16_OFFSET:].view(np.uint16)
    assert np.array_equal(bf[W.H_W3B:W.H_W3B + W.HID * W.HID],
                          I.to_bf16_bits(arr["W3b"].astype(np.float32)).reshape(-1))


def test_features_reproduce_the_cost():
    inst = I.c5(3)
    fs = W.features_np(inst.x, inst.y, inst.r, inst.cost_scale)
    ft = W.features_np(inst.y, inst.x, inst.c, inst.cost_scale)
    d2 = ((fs[:, None, :2] - ft[None, :, :2]) ** 2).sum(-1)
    assert np.max(np.abs(d2 - inst.C64)) <= 1e-12


def test_reference_is_permutation_equivariant_and_translation_invariant():
    arr = _random_weights(1)
    inst = I.c5(5)
    fs = W.features_np(inst.x, inst.y, inst.r, inst.cost_scale)
    ft = W.features_np(inst.y, inst.x, inst.c, inst.cost_scale)
    ps, pt = W.reference_predict(arr, fs, ft)
    perm = np.random.default_rng(2).permutation(inst.n)
    ps2, pt2 = W.reference_predict(arr, fs[perm], ft)
    assert np.allclose(ps2, ps[perm], rtol=1e-5, atol=1e-6)
    assert np.allclose(pt2, pt, rtol=1e-5, atol=1e-6)
    shift = np.array([0.37, -1.2])
    fs3 = W.features_np(inst.x + shift, inst.y + shift, inst.r, inst.cost_scale)
    ft3 = W.features_np(inst.y + shift, inst.x + shift, inst.c, inst.cost_scale)
    assert np.max(np.abs(fs3 - fs)) <= 1e-9 and np.max(np.abs(ft3 - ft)) <= 1e-9


def test_zero_mass_feature_is_clipped():
    inst = I.c5(7)
    r = inst.r.copy()
    r[4] = 0.0
    f = W.features_np(inst.x, inst.y, r, inst.cost_scale)
    assert f[4, 2] == -30.0 and np.all(np.isfinite(f))
