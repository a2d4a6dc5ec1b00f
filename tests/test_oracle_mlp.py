"""Pins of the oracle of the learned curvature (network arithmetic, BF16
rounding, backward pass, Adam, stencil canonicalisation).

The network is not in the paper, which computes curvature with height
functions; these tests pin the oracle to facts fixed independently of its
code: torch's own FP32 -> BF16 conversion, hand-built networks with known
outputs, central finite differences of the loss, closed forms of Adam's first
steps, and the symmetry group of the cube.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2407_07463_amd import synth

from mlp_fixtures import NP, OFF, random_inputs, random_params


# ------------------------------------------------------------------ BF16

def test_bf16_matches_torch_conversion():
    rng = synth.Splitmix64(11)
    v = np.concatenate([
        (rng.normal(20000) * 10.0 ** rng.uniform(20000).__mul__(12).__sub__(6)),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-40, 2.0 ** -126, 65504.0]),
    ]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16(v)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_bf16_ties_round_to_even():
    one = 1.0
    # representable neighbours of 1 are spaced 2^-7; halfway cases go to the even significand
    cases = [(one + 2.0 ** -8, one), (one + 3 * 2.0 ** -8, one + 2.0 ** -6), (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),
             (-(one + 2.0 ** -8), -one), (0.3, 0.30078125)]
    for v, want in cases:
        assert float(oracle.bf16([v])[0]) == want, v


# ------------------------------------------------------------------ forward

def _selector_network(w_centre=1.0, b3=0.25):
    P = np.zeros(NP, dtype=np.float32)
    P[OFF["W1"] + 13 * 128 + 0] = w_centre  # unit 0 of layer 1 reads the centre
    P[OFF["W2"] + 0 * 128 + 5] = 1.0        # unit 5 of layer 2 reads unit 0
    P[OFF["W3"] + 5] = 1.0
    P[OFF["b3"]] = b3
    return P


def test_forward_selector_network_rounding_points():
    x = np.zeros((3, 27), dtype=np.float32)
    x[0, 13] = 1.0 + 2.0 ** -8     # hi = 1, lo = 2^-8; the first activation rounds it back to 1
    x[1, 13] = 0.3
    x[2, 13] = 0.7
    x[2, 0] = 0.9                  # not connected
    y, acts = oracle.mlp_forward(_selector_network(), x)
    assert y.tolist() == [1.25, 0.25 + 0.30078125, 0.25 + 0.69921875]
    assert acts[1, 0] == 0.30078125 and acts[1, 128 + 5] == 0.30078125
    ye, _ = oracle.mlp_forward(_selector_network(), x, exact=True)
    assert ye[0] == 0.25 + (1.0 + 2.0 ** -8)


def test_forward_inputs_carry_sixteen_bits():
    # unit 0 of layer 1 takes the difference of two inputs that BF16 alone cannot tell apart
    P = _selector_network(b3=0.0)
    P[OFF["W1"] + 12 * 128 + 0] = -1.0
    x = np.zeros((2, 27), dtype=np.float32)
    x[:, 13] = 1.0 + 2.0 ** -8
    x[:, 12] = 1.0
    x[1, 13] = 1.0 + 2.0 ** -8 + 2.0 ** -15  # hi = 1 + 2^-7 (round up), lo = -2^-8 + 2^-15
    y, acts = oracle.mlp_forward(P, x)
    assert acts[0, 0] == 2.0 ** -8 and y[0] == 2.0 ** -8
    assert y[1] == float(oracle.bf16([2.0 ** -8 + 2.0 ** -15])[0])


def test_forward_last_layer_fp32():
    P = _selector_network(b3=0.0)
    P[OFF["b2"] + 5] = 2.0 ** -12          # second activation 1 + 2^-12: not rounded
    P[OFF["W3"] + 5] = 1.0 + 2.0 ** -10    # W3 in FP32: not rounded
    x = np.zeros((1, 27), dtype=np.float32)
    x[0, 13] = 1.0
    y, acts = oracle.mlp_forward(P, x)
    assert acts[0, 128 + 5] == 1.0 + 2.0 ** -12
    assert y[0] == (1.0 + 2.0 ** -12) * np.float64(np.float32(1.0 + 2.0 ** -10))


def test_forward_relu_cuts_negative_units():
    x = np.full((2, 27), 0.5, dtype=np.float32)
    y, acts = oracle.mlp_forward(_selector_network(w_centre=-1.0, b3=0.125), x)
    assert y.tolist() == [0.125, 0.125]
    assert acts[0, 256] == -0.5 and acts[0, 0] == 0.0


def test_forward_exact_matches_torch_float64():
    P = random_params(3)
    x = random_inputs(4, 64)
    y, acts = oracle.mlp_forward(P, x, exact=True)
    T = torch.from_numpy(P.astype(np.float64))
    W1 = T[OFF["W1"]:OFF["b1"]].reshape(32, 128)[:27]
    W2 = T[OFF["W2"]:OFF["b2"]].reshape(128, 128)
    X = torch.from_numpy(x.astype(np.float64))
    h1 = torch.relu(X @ W1 + T[OFF["b1"]:OFF["W2"]])
    h2 = torch.relu(h1 @ W2 + T[OFF["b2"]:OFF["W3"]])
    yr = h2 @ T[OFF["W3"]:OFF["b3"]] + T[OFF["b3"]]
    assert np.allclose(y, yr.numpy(), rtol=1e-13, atol=1e-13)
    assert np.allclose(acts[:, :128], h1.numpy(), rtol=1e-13, atol=1e-13)


def test_forward_bf16_matches_torch_rounding_points():
    P = random_params(5)
    x = random_inputs(6, 64)
    y, acts = oracle.mlp_forward(P, x)

    def b(t):  # via torch's own conversion
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    T = torch.from_numpy(P.astype(np.float64))
    W1 = b(T[OFF["W1"]:OFF["b1"]].reshape(32, 128)[:27])
    W2 = b(T[OFF["W2"]:OFF["b2"]].reshape(128, 128))
    W3 = T[OFF["W3"]:OFF["b3"]]
    X = torch.from_numpy(x)
    hi = X.to(torch.bfloat16).to(torch.float32)
    lo = (X - hi).to(torch.bfloat16).to(torch.float32)
    Xs = hi.to(torch.float64) + lo.to(torch.float64)
    assert torch.all((Xs - X.to(torch.float64)).abs() <= 2.0 ** -16 * X.abs().to(torch.float64))
    h1 = b(torch.relu(Xs @ W1 + T[OFF["b1"]:OFF["W2"]]))
    h2 = torch.relu(h1 @ W2 + T[OFF["b2"]:OFF["W3"]])
    yr = (h2 @ W3 + T[OFF["b3"]]).numpy()
    # summation order may move a rare pre-activation across a rounding boundary
    assert np.mean(acts[:, :128] != h1.numpy()) < 2e-3
    scale = (h2.abs() @ W3.abs()).numpy()
    assert np.all(np.abs(y - yr) <= 2e-3 * scale + 1e-12)
    assert np.median(np.abs(y - yr)) <= 1e-12


def test_layers_compose_to_forward():
    P = random_params(7)
    x = random_inputs(8, 16)
    y, acts = oracle.mlp_forward(P, x)
    _, a1, _ = oracle.mlp_layer(P, 1, x.astype(np.float64))
    _, a2, _ = oracle.mlp_layer(P, 2, a1)
    y3, _, _ = oracle.mlp_layer(P, 3, a2)
    assert np.array_equal(a1, acts[:, :128]) and np.array_equal(a2, acts[:, 128:256])
    assert np.allclose(y3, y, rtol=1e-15, atol=1e-15)


# ------------------------------------------------------------------ backward

def _loss_exact(P, x, t):
    y, _ = oracle.mlp_forward(P, x, exact=True)
    w = 1.0 / np.maximum(np.abs(t.astype(np.float64)), 0.05) ** 2
    return float(np.mean((y - t) ** 2 * w))


def test_backward_exact_matches_central_differences():
    P = random_params(9)
    x = random_inputs(10, 6)
    t = np.array([0.3, -0.2, 0.01, 0.5, -0.04, 0.15], dtype=np.float32)
    loss, g = oracle.mlp_grad(P, x, t, exact=True)
    assert abs(loss - _loss_exact(P, x, t)) <= 1e-14 * max(1.0, loss)
    rng = synth.Splitmix64(12)
    idx = np.concatenate([
        OFF["W1"] + (rng.uniform(40) * 27 * 128).astype(int),
        OFF["b1"] + (rng.uniform(20) * 128).astype(int),
        OFF["W2"] + (rng.uniform(60) * 128 * 128).astype(int),
        OFF["b2"] + (rng.uniform(20) * 128).astype(int),
        OFF["W3"] + (rng.uniform(20) * 128).astype(int),
        [OFF["b3"]],
    ])
    checked = 0
    for i in idx:
        h = np.float32(2.0 ** -12)
        Pp, Pm = P.copy(), P.copy()
        Pp[i] = P[i] + h
        Pm[i] = P[i] - h
        step = float(Pp[i]) - float(Pm[i])
        fd = (_loss_exact(Pp, x, t) - _loss_exact(Pm, x, t)) / step
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 1e-7 * max(1.0, loss), (i, fd, g[i])
        checked += abs(g[i]) > 1e-6
    assert checked > 50


def test_backward_rounded_close_to_exact_and_consistent():
    P = random_params(13)
    x = random_inputs(14, 32)
    t = (synth.Splitmix64(15).uniform(32) - 0.5).astype(np.float32)
    le, ge = oracle.mlp_grad(P, x, t, exact=True)
    lr_, gr = oracle.mlp_grad(P, x, t)
    assert abs(lr_ - le) <= 0.05 * le
    assert np.linalg.norm(gr - ge) <= 0.05 * np.linalg.norm(ge)
    # the same quantities through the layer-wise functions
    y, acts = oracle.mlp_forward(P, x)
    w = 1.0 / np.maximum(np.abs(t.astype(np.float64)), 0.05) ** 2
    g = 2.0 * (y - t) * w / len(t)
    h1, h2 = acts[:, :128], acts[:, 128:256]
    b = oracle.mlp_backward_given(P, x, g, h1, h2, np.zeros_like(h1), np.zeros_like(h1))
    b2 = oracle.mlp_backward_given(P, x, g, h1, h2, b["dz2"], np.zeros_like(h1))
    b3 = oracle.mlp_backward_given(P, x, g, h1, h2, b["dz2"], b2["dz1"])
    assert np.allclose(b3["grad"], gr, rtol=1e-12, atol=1e-15)
    assert np.all(b3["grad_abs"] >= np.abs(b3["grad"]) - 1e-15)


# ------------------------------------------------------------------ Adam

def test_adam_first_steps_closed_form():
    rng = synth.Splitmix64(16)
    P = rng.normal(NP).astype(np.float32)
    g = rng.normal(NP) * 10.0 ** (rng.uniform(NP) * 6 - 5)
    M = np.zeros(NP, dtype=np.float32)
    V = np.zeros(NP, dtype=np.float32)
    lr = 1e-3
    P1, M1, V1 = oracle.adam(P, M, V, g, 1, lr)
    # bias-corrected moments equal g and g^2 on the first step
    want = P.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.all(np.abs(P1 - want) <= 1e-7 * np.abs(want) + 1e-9)
    # a constant gradient: the bias-corrected moments stay g and g^2 on the second step
    P2, _, _ = oracle.adam(P1, M1, V1, g, 2, lr)
    want2 = P1.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.all(np.abs(P2 - want2) <= 1e-6 * lr + 1e-7 * np.abs(want2))
    # a zero gradient after one step: the first moment decays with beta1
    P2z, M2z, V2z = oracle.adam(P1, M1, V1, np.zeros(NP), 2, lr)
    assert np.allclose(M2z, 0.9 * M1, rtol=1e-6) and np.allclose(V2z, 0.999 * V1, rtol=1e-6)


# ------------------------------------------------------------------ canonicalisation

def _sphere_blocks(n, seed):
    """3x3x3 blocks around mixed cells of spheres of various radii."""
    rng = synth.Splitmix64(seed)
    blocks = []
    while len(blocks) < n:
        R = 2.0 + 10.0 * rng.uniform(1)[0]
        L = int(2 * R + 8)
        ctr = np.array([L / 2.0] * 3) + rng.uniform(3)
        c = synth.fill_spheres((L, L, L), 1, ctr[None], [R], [0])[0]
        mixed = np.argwhere((c > 0.0) & (c < 1.0))
        for q in (rng.uniform(4) * len(mixed)).astype(int):
            k, j, i = mixed[q]
            blocks.append(np.take(np.take(np.take(c, range(k - 1, k + 2), 0, mode="wrap"),
                                          range(j - 1, j + 2), 1, mode="wrap"), range(i - 1, i + 2), 2, mode="wrap"))
    return blocks[:n]


def _symmetries():
    out = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product([False, True], repeat=3):
            out.append((perm, flips))
    return out


def _apply(block, perm, flips):
    b = np.transpose(block, perm)
    for ax in range(3):
        if flips[ax]:
            b = np.flip(b, ax)
    return np.ascontiguousarray(b)


def _generic(block):
    m, _ = oracle.myc_normal(block)
    a = np.sort(np.abs(m))
    return a[0] > 1e-3 and a[1] - a[0] > 1e-3 and a[2] - a[1] > 1e-3 and abs(block[1, 1, 1] - 0.5) > 1e-3


def test_canonical_stencil_invariant_under_cube_group():
    syms = _symmetries()
    assert len(syms) == 48
    tested = 0
    for block in _sphere_blocks(60, 17):
        if not _generic(block):
            continue
        ref, s = oracle.canonical_stencil(block)
        for perm, flips in syms:
            got, s2 = oracle.canonical_stencil(_apply(block, perm, flips))
            assert s2 == s and np.array_equal(got, ref), (perm, flips)
        tested += 1
    assert tested >= 30


def test_canonical_stencil_form():
    n_flip = 0
    for block in _sphere_blocks(60, 18):
        if not _generic(block):
            continue
        x, s = oracle.canonical_stencil(block)
        src = block if s > 0 else 1.0 - block
        # the values are those of the block (complemented when the sign is -1), rearranged
        assert np.array_equal(np.sort(x), np.sort(src.astype(np.float32).ravel()))
        assert x[13] <= 0.5 and (s < 0) == (block[1, 1, 1] > 0.5)
        # the canonical block is one of the 48 images of src
        images = [_apply(src, p, f).astype(np.float32).ravel() for p, f in _symmetries()]
        assert any(np.array_equal(x, im) for im in images)
        m, _ = oracle.myc_normal(x.reshape(3, 3, 3).astype(np.float64))
        assert np.all(m >= -1e-6) and m[0] <= m[1] + 1e-6 <= m[2] + 2e-6
        n_flip += s < 0
    assert n_flip > 0


def test_canonical_stencil_phase_exchange_flips_sign():
    for block in _sphere_blocks(30, 19):
        if not _generic(block):
            continue
        x, s = oracle.canonical_stencil(block)
        xc, sc = oracle.canonical_stencil(1.0 - block)
        assert sc == -s
        assert np.allclose(xc, x, atol=2e-7, rtol=0)
