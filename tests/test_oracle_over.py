"""Pins of the oracle's ordered "over" compositing and of its adjoint.

Independent facts used: the hand-worked dyadic pixel, the front-to-back sum
form out = sum_i T_i L_i (a different formula for the same quantity), special
cases with closed forms, the FP32 tree-versus-sequential agreement the method
must keep (1e-6), and central finite differences (exact up to rounding, since
the loss is quadratic in every single input scalar)."""
import numpy as np
import pytest

import oracle
from conftest import read_golden


def _golden_layers():
    g = read_golden("over_1px.txt")
    rows = {r[0]: [float(v) for v in r[1:]] for r in g["layers_back_to_front"]}
    names = ["far", "mid", "near"]
    layers = [np.array(rows[k], np.float64).reshape(1, 1, 4) for k in names]
    return g, names, layers


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.float16])
def test_worked_example(dtype):
    g, names, layers = _golden_layers()
    layers = [l.astype(dtype) for l in layers]
    exp = np.array([float(v) for v in g["out"][0]])
    rois = [(0, 0, 1, 1)] * 3
    out = oracle.composite_over(layers, rois, [0, 1, 2], (0, 0, 1, 1))
    assert (out[0, 0] == exp).all()
    for P in (1, 2):
        t = oracle.composite_over(layers, rois, [0, 1, 2], (0, 0, 1, 1), groups=P)
        assert (t[0, 0] == exp).all()
        f = oracle.composite_over_f32(layers, rois, [0, 1, 2], (0, 0, 1, 1), groups=P)
        assert (f[0, 0] == exp.astype(np.float32)).all()
    # the front pair of the two-group tree
    pair = oracle.composite_over(layers[1:], rois[1:], [0, 1], (0, 0, 1, 1))
    assert (pair[0, 0] == np.array([float(v) for v in g["tree_front_pair"][0]])).all()


def test_worked_example_adjoint():
    g, names, layers = _golden_layers()
    out = oracle.composite_over(layers, [(0, 0, 1, 1)] * 3, [0, 1, 2], (0, 0, 1, 1))
    G = np.zeros((1, 1, 4))
    G[0, 0, 0] = 2 * (out[0, 0, 0] - 0.5)
    assert G[0, 0, 0] == 0.3125
    grads = oracle.composite_over_backward(layers, [(0, 0, 1, 1)] * 3, [0, 1, 2], (0, 0, 1, 1), G)
    gc = {r[0]: float(r[1]) for r in g["grad_c"]}
    ga = {r[0]: float(r[1]) for r in g["grad_alpha"]}
    for i, nm in enumerate(names):
        assert grads[i][0, 0, 0] == gc[nm]
        assert grads[i][0, 0, 3] == ga[nm]
        assert grads[i][0, 0, 1] == 0 and grads[i][0, 0, 2] == 0


def test_worked_example_adjoint_scale():
    """The componentwise condition scale that every GPU backward tolerance is
    multiplied by, pinned to hand-worked values: with G >= 0 (nothing
    cancels), and with a mixed-sign G whose alpha terms partly cancel."""
    g, names, layers = _golden_layers()
    rois, vp = [(0, 0, 1, 1)] * 3, (0, 0, 1, 1)
    G = np.zeros((1, 1, 4))
    G[0, 0, 0] = 0.3125
    _, scale = oracle.composite_over_backward(layers, rois, [0, 1, 2], vp, G, want_scale=True)
    sc = {r[0]: float(r[1]) for r in g["gscale_c"]}
    sa = {r[0]: float(r[1]) for r in g["gscale_alpha"]}
    for i, nm in enumerate(names):
        assert scale[i][0, 0, 0] == sc[nm]
        assert scale[i][0, 0, 3] == sa[nm]
        assert scale[i][0, 0, 1] == 0 and scale[i][0, 0, 2] == 0
    G[0, 0, 3] = -0.5
    grads, scale = oracle.composite_over_backward(layers, rois, [0, 1, 2], vp, G, want_scale=True)
    gam = {r[0]: float(r[1]) for r in g["grad_alpha_mixed"]}
    sam = {r[0]: float(r[1]) for r in g["gscale_alpha_mixed"]}
    for i, nm in enumerate(names):
        assert grads[i][0, 0, 0] == sc[nm]   # G_0 >= 0: |grad c| = its scale
        assert grads[i][0, 0, 3] == gam[nm]
        assert scale[i][0, 0, 3] == sam[nm]
        # the scale bounds the gradient's own magnitude
        assert abs(grads[i][0, 0, 3]) <= scale[i][0, 0, 3]


def _rand_layers(rng, n, W, H, full=False, dtype=np.float64):
    layers, rois = [], []
    for _ in range(n):
        if full:
            x, y, w, h = 0, 0, W, H
        else:
            w, h = int(rng.integers(1, W + 1)), int(rng.integers(1, H + 1))
            x, y = int(rng.integers(-1, W)), int(rng.integers(-1, H))
        P = w + int(rng.integers(0, 3))
        a = rng.beta(2, 5, size=(h, P))
        L = np.empty((h, P, 4))
        L[..., :3] = rng.random((h, P, 3)) * a[..., None]
        L[..., 3] = a
        layers.append(L.astype(dtype))
        rois.append((x, y, w, h))
    return layers, rois


def _front_to_back_sum(layers, rois, order, vp):
    """out = sum_i T_i L_i with T_0 = 1, T_{i+1} = T_i (1 - a_i), i = 0 nearest."""
    X0, Y0, W, H = vp
    out = np.zeros((H, W, 4))
    T = np.ones((H, W))
    for li in reversed(order):
        x, y, w, h = rois[li]
        L = np.zeros((H, W, 4))
        for v in range(H):
            for u in range(W):
                X, Y = X0 + u, Y0 + v
                if x <= X < x + w and y <= Y < y + h:
                    L[v, u] = layers[li][Y - y, X - x]
        out += T[..., None] * L
        T = T * (1 - L[..., 3])
    return out


@pytest.mark.parametrize("seed", range(6))
def test_back_to_front_equals_front_to_back_sum(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    layers, rois = _rand_layers(rng, n, 7, 5)
    order = list(rng.permutation(n))
    vp = (0, 0, 7, 5)
    a = oracle.composite_over(layers, rois, order, vp)
    b = _front_to_back_sum(layers, rois, order, vp)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16])
def test_tree_orders(P):
    rng = np.random.default_rng(40 + P)
    n = 13
    layers, rois = _rand_layers(rng, n, 9, 6)
    order = list(rng.permutation(n))
    vp = (0, 0, 9, 6)
    seq = oracle.composite_over(layers, rois, order, vp)
    tree = oracle.composite_over(layers, rois, order, vp, groups=P)
    assert np.allclose(tree, seq, rtol=1e-14, atol=1e-300)
    # single precision: tree and sequential agree within 1e-6 (relative)
    l32 = [l.astype(np.float32) for l in layers]
    s32 = oracle.composite_over_f32(l32, rois, order, vp, groups=1)
    t32 = oracle.composite_over_f32(l32, rois, order, vp, groups=P)
    assert (np.abs(t32.astype(np.float64) - s32) <= 1e-6 * np.abs(s32) + 1e-30).all()
    # and the FP32 sequential order is within 2e-6 of the FP64 result of the
    # same (fp32-stored) inputs
    ref = oracle.composite_over(l32, rois, order, vp)
    assert (np.abs(s32 - ref) <= 2e-6 * np.abs(ref) + 1e-30).all()


def test_fp32_tree_vs_sequential_many_layers():
    """64 full-frame layers as in the 3840x2160 brick workload, on a patch."""
    rng = np.random.default_rng(5)
    layers, rois = _rand_layers(rng, 64, 16, 16, full=True, dtype=np.float32)
    order = list(rng.permutation(64))
    vp = (0, 0, 16, 16)
    s32 = oracle.composite_over_f32(layers, rois, order, vp, groups=1)
    for P in (2, 4, 8, 16, 64):
        t32 = oracle.composite_over_f32(layers, rois, order, vp, groups=P)
        assert (np.abs(t32.astype(np.float64) - s32) <= 1e-6 * np.abs(s32) + 1e-30).all()


def test_special_cases():
    rng = np.random.default_rng(9)
    layers, rois = _rand_layers(rng, 5, 6, 4, full=True)
    vp = (0, 0, 6, 4)
    order = [3, 1, 4, 0, 2]
    # n = 1 is the identity
    one = oracle.composite_over(layers[:1], rois[:1], [0], vp)
    assert (one == layers[0][:, :6]).all()
    # all alpha = 1: exactly the front-most layer
    opaque = [l.copy() for l in layers]
    for l in opaque:
        l[..., 3] = 1.0
    out = oracle.composite_over(opaque, rois, order, vp)
    assert (out == opaque[order[-1]][:, :6]).all()
    # all zero: zero
    zeros = [np.zeros_like(l) for l in layers]
    assert (oracle.composite_over(zeros, rois, order, vp) == 0).all()
    # a zero layer anywhere is the identity element (bitwise)
    base = oracle.composite_over(layers, rois, order, vp)
    for pos in range(6):
        l2 = layers + [np.zeros_like(layers[0])]
        o2 = order[:pos] + [5] + order[pos:]
        assert (oracle.composite_over(l2, rois + [rois[0]], o2, vp) == base).all()
    # all alpha = 0: the plain sum of the colours
    clear = [l.copy() for l in layers]
    for l in clear:
        l[..., 3] = 0.0
    out = oracle.composite_over(clear, rois, order, vp)
    assert np.allclose(out, sum(l[:, :6] for l in clear), rtol=1e-15, atol=0)
    # a layer outside the viewport contributes nothing
    far = oracle.composite_over(layers[:1], [(100, 100, 6, 4)], [0], vp)
    assert (far == 0).all()


def _pixel_loss(layers, rois, order, X, Y, target):
    out = oracle.composite_over(layers, rois, order, (X, Y, 1, 1))[0, 0]
    return float(((out - target) ** 2).sum())


@pytest.mark.parametrize("seed", range(4))
def test_adjoint_matches_central_differences(seed):
    """loss = sum (out - t)^2 is a quadratic polynomial of any one input
    scalar, so the central difference with h = 1e-3 is exact up to rounding."""
    rng = np.random.default_rng(70 + seed)
    n = int(rng.integers(1, 7))
    W, H = 5, 4
    layers, rois = _rand_layers(rng, n, W, H)
    order = list(rng.permutation(n))
    vp = (0, 0, W, H)
    target = rng.random((H, W, 4))
    out = oracle.composite_over(layers, rois, order, vp)
    G = 2 * (out - target)
    grads, scales = oracle.composite_over_backward(layers, rois, order, vp, G, want_scale=True)
    h = 1e-3
    checked = 0
    for i in range(n):
        x, y, w, hh = rois[i]
        for yy in range(hh):
            for xx in range(w):
                X, Y = x + xx, y + yy
                inside = 0 <= X < W and 0 <= Y < H
                for k in range(4):
                    if not inside:
                        assert grads[i][yy, xx, k] == 0.0
                        continue
                    lp = [l.copy() for l in layers]
                    lm = [l.copy() for l in layers]
                    lp[i][yy, xx, k] += h
                    lm[i][yy, xx, k] -= h
                    fd = (_pixel_loss(lp, rois, order, X, Y, target[Y, X])
                          - _pixel_loss(lm, rois, order, X, Y, target[Y, X])) / (2 * h)
                    assert abs(fd - grads[i][yy, xx, k]) <= 2e-11, (i, yy, xx, k)
                    checked += 1
    assert checked > 0
    for s in scales:
        assert (s >= 0).all()


def test_adjoint_special_cases():
    rng = np.random.default_rng(12)
    layers, rois = _rand_layers(rng, 4, 3, 3, full=True)
    vp = (0, 0, 3, 3)
    G = rng.standard_normal((3, 3, 4))
    # n = 1: the gradient is G
    g1 = oracle.composite_over_backward(layers[:1], rois[:1], [0], vp, G)
    assert (g1[0][:, :3] == G).all()
    # an opaque layer hides everything behind it: zero gradient there
    order = [0, 1, 2, 3]          # back to front; layer 2 is second nearest
    layers[2][..., 3] = 1.0
    g = oracle.composite_over_backward(layers, rois, order, vp, G)
    assert (g[0] == 0).all() and (g[1] == 0).all()
    assert (g[3][:, :3, :3] == G[..., :3]).all()
