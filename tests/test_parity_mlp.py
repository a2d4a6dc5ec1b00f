"""GPU parity of the learned curvature (forward, training step, stencils,
combined curvature) against the CPU oracle, through the C ABI.

Bars:
- stencils, cells and signs bit-exact (same FP64 decisions, exact FP32 casts);
- each layer, fed the GPU's own rounded inputs, within the FP32 accumulation
  bound K * 2^-23 * sum |a b| of the oracle's FP64 value, plus one BF16 ulp
  where a rounded activation sits at a rounding boundary;
- backward quantities likewise, on the GPU's own intermediates (trace);
- Adam within FP32 rounding of the FP64 update;
- combined curvature: exactly the height-function value or sign * network
  output, chosen by the stated rule.
"""
import numpy as np
import pytest

import oracle
from gpu_util import note, require_gpu
from mlp_fixtures import NP, OFF, canonical_inputs, random_inputs, random_params, sphere_field
from paper_2407_07463_amd import synth

pytestmark = pytest.mark.gpu

U23 = 2.0 ** -23
BF_ULP = 2.0 ** -7  # relative spacing of BF16 at worst


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    from paper_2407_07463_amd import vofmt

    c = vofmt.Context(0)
    yield c
    c.close()
    del torch


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _bf(u16):
    """BF16 bit patterns -> float64."""
    return (np.asarray(u16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _records(rec):
    """Activation / training records (bytes) -> h1, h2[, dz2, dz1] as float64."""
    rec = np.ascontiguousarray(rec)
    h1 = _bf(rec[:, 0:256].view(np.uint16))
    h2 = rec[:, 256:768].view(np.float32).astype(np.float64)
    if rec.shape[1] == 768:
        return h1, h2
    return h1, h2, _bf(rec[:, 768:1024].view(np.uint16)), _bf(rec[:, 1024:1280].view(np.uint16))


def _check_fp32(got, ref, absacc, K, what):
    ok = np.abs(got - ref) <= K * U23 * absacc + 1e-30
    assert ok.all(), (what, np.argwhere(~ok)[:5], got[~ok][:5], ref[~ok][:5])


def _check_rounded(got, ref, absacc, K, what):
    """A rounded activation: FP32 accumulation bound, plus one BF16 ulp at a boundary."""
    bound = K * U23 * absacc
    err = np.abs(got - ref)
    ok = err <= BF_ULP * np.abs(ref) + 2 * bound + 1e-30
    assert ok.all(), (what, np.argwhere(~ok)[:5], got[~ok][:5], ref[~ok][:5])
    # boundary cases are rare
    assert np.mean(err > bound * 2 + 1e-30) < 0.02, what


def _mixed_inputs(n_sphere_fields=3, seed=100):
    xs = []
    for q in range(n_sphere_fields):
        R = [2.5, 5.0, 9.0][q % 3]
        _, x, _ = canonical_inputs(sphere_field(R, seed + q, drop=(q % 2 == 0)))
        xs.append(x)
    return np.concatenate(xs)


@pytest.mark.parametrize("m,kind", [(1, "uniform"), (64, "uniform"), (203, "uniform"), (0, "uniform"),
                                    (1000, "spheres"), (40000, "uniform")])
def test_forward_layers(ctx, m, kind):
    import torch

    P = random_params(21)
    if kind == "spheres":
        x = _mixed_inputs()[:m]
        m = len(x)
    else:
        x = random_inputs(22 + m, m) if m else np.zeros((0, 27), np.float32)
    note(f"mlp forward m={m} kind={kind}")
    Pd, xd = _dev(P), _dev(x)
    y = torch.zeros(max(m, 1), dtype=torch.float32, device="cuda:0")
    acts = torch.zeros((max(m, 1), 768), dtype=torch.uint8, device="cuda:0")
    ctx.mlp_forward(Pd, xd, y, acts)
    torch.cuda.synchronize()
    if m == 0:
        return
    y, acts = y.cpu().numpy()[:m], acts.cpu().numpy()[:m]
    h1, h2 = _records(acts)
    _, a1, ab1 = oracle.mlp_layer(P, 1, x.astype(np.float64))
    _check_rounded(h1, a1, ab1, 64, "h1")
    _, a2, ab2 = oracle.mlp_layer(P, 2, h1)
    _check_fp32(h2, a2, ab2, 129, "h2")
    y3, _, ab3 = oracle.mlp_layer(P, 3, h2)
    assert np.all(np.abs(y - y3) <= (128 + 8) * U23 * ab3 + 1e-30)
    # end to end against the oracle's own forward pass: same up to rare boundary flips
    yo, _ = oracle.mlp_forward(P, x)
    assert np.median(np.abs(y - yo) / np.maximum(np.abs(yo), 1e-3)) < 1e-4


def test_forward_rejects_bad_arguments(ctx):
    import torch

    from paper_2407_07463_amd import vofmt

    P = _dev(random_params(1))
    x = torch.zeros((4, 27), dtype=torch.float32, device="cuda:0")
    y = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    L = vofmt.load()
    rc = L.vofmt_mlp_forward(ctx.h, vofmt._ptr(P), -1, vofmt._ptr(x), vofmt._ptr(y), None, vofmt._stream())
    assert rc == vofmt.E_ARG
    with pytest.raises(vofmt.VofmtError):
        ctx.mlp_train_step(P, torch.zeros_like(P), torch.zeros_like(P), 0, 1e-3, x, y)


@pytest.mark.parametrize("m,step", [(203, 1), (64, 1), (1, 1), (4096, 3)])
def test_train_step(ctx, m, step):
    import torch

    P = random_params(31)
    rng = synth.Splitmix64(32 + m)
    x = random_inputs(33 + m, m)
    t = ((rng.uniform(m) - 0.5) * 0.8).astype(np.float32)
    t[: m // 10] = 0.01  # small targets: the loss weight saturates at 1/0.05^2
    M0 = (rng.normal(NP) * 1e-3).astype(np.float32) if step > 1 else np.zeros(NP, np.float32)
    V0 = (np.abs(rng.normal(NP)) * 1e-6).astype(np.float32) if step > 1 else np.zeros(NP, np.float32)
    lr = 1e-3
    note(f"mlp train step m={m} step={step}")
    Pd, Md, Vd = _dev(P), _dev(M0), _dev(V0)
    y = torch.zeros(m, dtype=torch.float32, device="cuda:0")
    acts = torch.zeros((m, 768), dtype=torch.uint8, device="cuda:0")
    ctx.mlp_forward(Pd, _dev(x), y, acts)
    grads = torch.zeros(NP, dtype=torch.float32, device="cuda:0")
    trace = torch.zeros((m, 1280), dtype=torch.uint8, device="cuda:0")
    loss = ctx.mlp_train_step(Pd, Md, Vd, step, lr, _dev(x), _dev(t), grads, trace)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    acts = acts.cpu().numpy()
    tr = trace.cpu().numpy()
    G = grads.cpu().numpy().astype(np.float64)
    P1, M1, V1 = Pd.cpu().numpy(), Md.cpu().numpy(), Vd.cpu().numpy()
    # the training forward pass is the inference forward pass
    assert np.array_equal(tr[:, :768], acts)
    h1, h2, dz2, dz1 = _records(tr)
    w = 1.0 / np.maximum(np.abs(t.astype(np.float64)), 0.05) ** 2
    lo = np.mean((y - t) ** 2 * w)
    assert abs(loss - lo) <= 2e-5 * lo + 1e-12
    g = 2.0 * (y - t) * w / m
    b = oracle.mlp_backward_given(P, x, g, h1, h2, dz2, dz1)
    ok2 = np.abs(dz2 - b["dz2"]) <= BF_ULP * np.abs(b["dz2"]) + 1e-30
    assert ok2.all()
    _check_rounded(dz1, b["dz1"], b["dz1_abs"], 128, "dz1")
    ntiles = (m + 63) // 64
    K = 128 + ntiles + 8  # dW1 sums hi and lo products: 2 x 64 per tile
    err = np.abs(G - b["grad"])
    ok = err <= K * U23 * b["grad_abs"] + 1e-30
    assert ok.all(), (np.argwhere(~ok)[:5], G[~ok][:5], b["grad"][~ok][:5])
    # padding rows of W1 see zero inputs
    assert np.all(G[OFF["W1"] + 27 * 128:OFF["b1"]] == 0.0)
    # Adam on the GPU's gradient
    Po, Mo, Vo = oracle.adam(P, M0, V0, G, step, lr)
    assert np.all(np.abs(P1.astype(np.float64) - Po) <= 1e-5 * lr + 2 * U23 * np.abs(Po))
    assert np.all(np.abs(M1.astype(np.float64) - Mo) <= 4 * U23 * (0.9 * np.abs(M0) + 0.1 * np.abs(G)) + 1e-38)
    assert np.all(np.abs(V1.astype(np.float64) - Vo) <= 4 * U23 * (0.999 * V0 + 0.001 * G * G) + 1e-38)


def test_train_step_reproducible(ctx):
    import torch

    P = random_params(41)
    x = random_inputs(42, 3000)
    t = (synth.Splitmix64(43).uniform(3000) * 0.5).astype(np.float32)
    outs = []
    for _ in range(2):
        Pd = _dev(P)
        Md = torch.zeros_like(Pd)
        Vd = torch.zeros_like(Pd)
        losses = [ctx.mlp_train_step(Pd, Md, Vd, s, 1e-3, _dev(x), _dev(t)) for s in (1, 2, 3)]
        torch.cuda.synchronize()
        outs.append((Pd.cpu().numpy(), losses))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
    assert outs[0][1][2] < outs[0][1][0]  # the loss goes down


@pytest.mark.parametrize("R,drop", [(2.5, True), (6.0, False), (11.0, True)])
def test_stencils_bit_exact(ctx, R, drop):
    import torch

    c = sphere_field(R, 50, drop)
    cells, xs, sg = canonical_inputs(c)
    n = len(cells)
    note(f"mlp stencils R={R} drop={drop} n={n}")
    xd = torch.zeros((n + 5, 27), dtype=torch.float32, device="cuda:0")
    cd = torch.zeros(n + 5, dtype=torch.int32, device="cuda:0")
    sd = torch.zeros(n + 5, dtype=torch.int8, device="cuda:0")
    got = ctx.mlp_stencils(_dev(c), xd, cd, sd)
    torch.cuda.synchronize()
    assert got == n
    assert np.array_equal(cd.cpu().numpy()[:n], cells)
    assert np.array_equal(sd.cpu().numpy()[:n], sg)
    assert np.array_equal(xd.cpu().numpy()[:n].view(np.uint32), xs.view(np.uint32))


def test_stencils_edge_cases(ctx):
    import torch

    from paper_2407_07463_amd import vofmt

    xd = torch.zeros((4, 27), dtype=torch.float32, device="cuda:0")
    cd = torch.zeros(4, dtype=torch.int32, device="cuda:0")
    sd = torch.zeros(4, dtype=torch.int8, device="cuda:0")
    for v in (0.0, 1.0):
        c = torch.full((5, 6, 7), v, dtype=torch.float64, device="cuda:0")
        assert ctx.mlp_stencils(c, xd, cd, sd) == 0
    c = _dev(sphere_field(3.0, 51))
    with pytest.raises(vofmt.VofmtError):
        ctx.mlp_stencils(c, xd, cd, sd)  # capacity 4 is too small


@pytest.mark.parametrize("R,kappa_lo", [(3.0, 0.3), (8.0, 0.3), (8.0, 0.0)])
def test_curvature_mlp_combination(ctx, R, kappa_lo):
    import torch

    P = random_params(61, scale=0.3)
    c = sphere_field(R, 62)
    cells, xs, sg = canonical_inputs(c)
    note(f"curvature mlp R={R} kappa_lo={kappa_lo}")
    cd = _dev(c)
    kap = torch.zeros(c.shape, dtype=torch.float64, device="cuda:0")
    st = torch.zeros(c.shape, dtype=torch.uint8, device="cuda:0")
    nm = ctx.curvature_mlp(cd, _dev(P), kappa_lo, kap, st)
    y = torch.zeros(len(cells), dtype=torch.float32, device="cuda:0")
    ctx.mlp_forward(_dev(P), _dev(xs), y)
    torch.cuda.synchronize()
    assert nm == len(cells)
    kap, st, y = kap.cpu().numpy().ravel(), st.cpu().numpy().ravel(), y.cpu().numpy().astype(np.float64)
    khf, shf = oracle.curvature_hf(c)
    khf, shf = khf.ravel(), shf.ravel()
    net = sg.astype(np.float64) * y
    # the network's value unless |kappa| < kappa_lo and the height function is valid there
    flag = np.abs(net) < kappa_lo
    hs = shf[cells]
    hf_ok = flag & (hs >= 1) & (hs <= 3)
    want_k = np.where(hf_ok, khf[cells], net)
    want_s = np.where(flag, np.where(hf_ok, hs, hs | 8), 8)
    assert np.array_equal(st[cells], want_s)
    assert np.array_equal(kap[cells], want_k)
    other = np.setdiff1d(np.arange(c.size), cells)
    assert np.all(st[other] == 0) and np.all(np.isnan(kap[other]))
    if kappa_lo == 0.0:
        assert np.all(st[cells] == 8)
