"""GPU parity of the learned curvature (forward, training step, stencils,
combined curvature) against the CPU oracle, through the C ABI.

Every oracle value is computed by the oracle from the test's own inputs: the
oracle runs the whole chain (x -> h1 -> h2 -> y, then dz2 -> dz1 -> gradient
-> Adam) in FP64 with the kernels' BF16 rounding points, and each GPU stage is
compared with the oracle's value of that stage.

Bars, stage by stage:
- stencils, cells and signs bit-exact (same FP64 decisions, exact FP32 casts);
- a stage within the FP32 accumulation bound K * 2^-23 * sum |a b| plus the
  deviation of its GPU inputs from the oracle's, carried through the layer
  (|W| times the input deviations; ReLU does not enlarge it); a rounded
  stage equal to a rounding of some value within that bound of the oracle's
  pre-activation (one BF16 ulp off only where the bound reaches a rounding
  midpoint), and a ReLU mask may differ only where the stage's bound reaches
  zero;
- Adam: the GPU update lies within the oracle's updates over the gradient's
  bound, up to FP32 rounding;
- combined curvature: the height-function value or sign * network output,
  chosen by the stated rule; a cell whose oracle output lies within the
  output bound of the threshold may take either branch.
"""
import numpy as np
import pytest

import oracle
from gpu_util import note, require_gpu
from mlp_fixtures import NP, OFF, block_at, canonical_inputs, random_inputs, random_params, sphere_field
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


def _bf16_vec(v):
    """FP32 -> BF16 -> FP32, round to nearest even (finite values), vectorised; checked against
    the oracle's scalar rounding on a sample of every call."""
    v32 = np.ascontiguousarray(v, dtype=np.float32)
    u = v32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    sample = v32.ravel()[:: max(1, v32.size // 64)]
    assert np.array_equal(oracle.bf16(sample), r.ravel()[:: max(1, v32.size // 64)])
    return r


def _check_rounded(got, pre, absacc, K, what):
    """A rounded activation bf16(relu(z)), z the FP32 accumulation of the oracle's pre-activation
    pre within K 2^-23 absacc: rounding is monotone, so the GPU's value must lie between the
    roundings of the two ends of that interval -- it may differ from the oracle's rounding only
    where the interval reaches a BF16 rounding midpoint (or zero)."""
    bound = K * U23 * absacc + np.abs(pre) * 2.0 ** -24  # and the FP32 rounding of the ends
    lo = _bf16_vec(np.maximum(pre - bound, 0.0)).astype(np.float64)
    hi = _bf16_vec(np.maximum(pre + bound, 0.0)).astype(np.float64)
    ok = (got >= lo) & (got <= hi)
    assert ok.all(), (what, np.argwhere(~ok)[:5], got[~ok][:5], pre[~ok][:5])


def _weights(P):
    """Weights as the network uses them: BF16 W1 [32][128] and W2 [128][128]
    (rows = inputs), FP32 W3 [128]."""
    W1 = oracle.bf16(P[OFF["W1"]:OFF["b1"]]).astype(np.float64).reshape(32, 128)
    W2 = oracle.bf16(P[OFF["W2"]:OFF["b2"]]).astype(np.float64).reshape(128, 128)
    W3 = P[OFF["W3"]:OFF["b3"]].astype(np.float64)
    return W1, W2, W3


def _check_carried(got, ref, absacc, carried, K, what):
    """FP32 accumulation over the GPU's inputs (scale absacc + carried) plus the
    deviation of those inputs from the oracle's, carried through the layer."""
    bound = K * U23 * (absacc + carried) + carried + 1e-30
    ok = np.abs(got - ref) <= bound
    assert ok.all(), (what, np.argwhere(~ok)[:5], got[~ok][:5], ref[~ok][:5])
    return bound


def _forward_chain(P, x, h1, h2, y):
    """The GPU's h1, h2, y against the oracle's chain on the same inputs x.
    Returns the oracle's h1, h2, y and the bound on |y - y_oracle|."""
    _, W2, W3 = _weights(P)
    pre1, h1o, ab1 = oracle.mlp_layer(P, 1, x.astype(np.float64))
    _check_rounded(h1, pre1, ab1, 64, "h1")
    _, h2o, ab2 = oracle.mlp_layer(P, 2, h1o)
    _check_carried(h2, h2o, ab2, np.abs(h1 - h1o) @ np.abs(W2), 129, "h2")
    yo, _, ab3 = oracle.mlp_layer(P, 3, h2o)
    ybound = _check_carried(y, yo, ab3, np.abs(h2 - h2o) @ np.abs(W3), 128 + 8, "y")
    return h1o, h2o, yo, ybound


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
    y, acts = y.cpu().numpy()[:m].astype(np.float64), acts.cpu().numpy()[:m]
    h1, h2 = _records(acts)
    _, _, y3, _ = _forward_chain(P, x, h1, h2, y)
    # the chain of single layers is the oracle's forward pass, and the GPU
    # output differs from it only where a BF16 rounding sits at a boundary
    yo, _ = oracle.mlp_forward(P, x)
    assert np.array_equal(y3, yo)
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


@pytest.mark.parametrize("m,step", [(203, 1), (64, 1), (1, 1), (4096, 3), (40000, 2)])
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
    h1o, h2o, yo, ybound = _forward_chain(P, x, h1, h2, y)
    _, W2, W3 = _weights(P)
    tt = t.astype(np.float64)
    w = 1.0 / np.maximum(np.abs(tt), 0.05) ** 2
    dy = np.abs(y - yo)
    # loss: FP32 sum, plus (y - t)^2 - (yo - t)^2 = dy (2 (yo - t) + dy)
    lo = np.mean((yo - tt) ** 2 * w)
    assert abs(loss - lo) <= 2e-5 * lo + np.mean(w * dy * (2 * np.abs(yo - tt) + dy)) + 1e-12
    go = 2.0 * (yo - tt) * w / m
    dg = 2.0 * dy * w / m + 4 * U23 * np.abs(go)
    # the oracle's backward chain on its own forward chain
    zero = np.zeros((m, 128))
    dz2o = oracle.mlp_backward_given(P, x, go, h1o, h2o, zero, zero)["dz2"]
    b = oracle.mlp_backward_given(P, x, go, h1o, h2o, dz2o, zero)
    dz1o, dz1abs = b["dz1"], b["dz1_abs"]
    b = oracle.mlp_backward_given(P, x, go, h1o, h2o, dz2o, dz1o)
    # dz2 = round(h2 > 0 ? g W3 : 0)
    a3 = np.abs(W3)[None, :]
    flip2 = (h2 > 0) != (h2o > 0)
    lim2 = np.where(flip2, (np.abs(go) + dg)[:, None] * a3, BF_ULP * np.abs(dz2o) + dg[:, None] * a3)
    ok = np.abs(dz2 - dz2o) <= lim2 * (1 + BF_ULP) + 1e-30
    assert ok.all(), ("dz2", np.argwhere(~ok)[:5])
    # dz1 = round(h1 > 0 ? sum_j dz2_j W2[k][j] : 0)
    c1 = np.abs(dz2 - dz2o) @ np.abs(W2).T
    flip1 = (h1 > 0) != (h1o > 0)
    acc1 = 2 * 128 * U23 * (dz1abs + c1) + c1
    lim1 = np.where(flip1, dz1abs + c1, BF_ULP * np.abs(dz1o) + acc1)
    ok = np.abs(dz1 - dz1o) <= lim1 * (1 + BF_ULP) + 1e-30
    assert ok.all(), ("dz1", np.argwhere(~ok)[:5])
    # gradient: FP32 sums over the batch of products whose factors carry the
    # deviations checked above
    dh1, dh2 = np.abs(h1 - h1o), np.abs(h2 - h2o)
    dd2, dd1 = np.abs(dz2 - dz2o), np.abs(dz1 - dz1o)
    xb = np.abs(x.astype(np.float64)) * (1 + 2.0 ** -15)  # hi + lo split of each input
    carried = np.zeros(NP)
    carried[OFF["W3"]:OFF["b3"]] = dg @ np.abs(h2o) + np.abs(go) @ dh2 + dg @ dh2
    carried[OFF["b3"]] = dg.sum()
    carried[OFF["W2"]:OFF["b2"]] = (dh1.T @ np.abs(dz2o) + np.abs(h1o).T @ dd2 + dh1.T @ dd2).ravel()
    carried[OFF["b2"]:OFF["W3"]] = dd2.sum(axis=0)
    carried[OFF["W1"]:OFF["W1"] + 27 * 128] = (xb.T @ dd1).ravel()
    carried[OFF["b1"]:OFF["W2"]] = dd1.sum(axis=0)
    ntiles = (m + 63) // 64
    # a workgroup per compute unit at most, each over T consecutive tiles: dW1 chains hi and lo
    # products, 2 x 64 per tile, then the partials of the groups are added
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    T = -(-ntiles // min(ntiles, cus))
    groups = -(-ntiles // T)
    K = 128 * T + groups + 8
    gbound = _check_carried(G, b["grad"], b["grad_abs"], carried, K, "grad")
    # padding rows of W1 see zero inputs
    assert np.all(G[OFF["W1"] + 27 * 128:OFF["b1"]] == 0.0)
    # Adam: m and v are affine and quadratic in the gradient; the update lies
    # within the oracle's updates over the gradient's bound
    go_all = b["grad"]
    Po, Mo, Vo = oracle.adam(P, M0, V0, go_all, step, lr)
    ag = np.abs(go_all) + gbound
    assert np.all(np.abs(M1.astype(np.float64) - Mo) <= 4 * U23 * (0.9 * np.abs(M0) + 0.1 * ag) + 0.1 * gbound
                  + 1e-38)
    assert np.all(np.abs(V1.astype(np.float64) - Vo) <= 4 * U23 * (0.999 * V0 + 0.001 * ag * ag)
                  + 0.001 * (2 * np.abs(go_all) + gbound) * gbound + 1e-38)
    outs = np.stack([oracle.adam(P, M0, V0, go_all + f * gbound, step, lr)[0].astype(np.float64)
                     for f in np.linspace(-1.0, 1.0, 11)])
    slack = 1e-5 * lr + 2 * U23 * np.abs(Po.astype(np.float64))
    P1d = P1.astype(np.float64)
    assert np.all(P1d >= outs.min(axis=0) - slack) and np.all(P1d <= outs.max(axis=0) + slack)


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


def _check_combined(kc, sc, khf, shf, sg, y, yo, ybound, kappa_lo, two):
    """Combined curvature of mixed cells (values kc, statuses sc) against the
    rule: the network's value sign * y, unless |sign * y| < kappa_lo or the
    block holds two interfaces (two, from the oracle) and the height function
    is valid there (status 1-3), then the height function's value; status 8
    marks a network value, 8 | s one whose height function (status s) was
    wanted but not valid. y: the GPU network outputs on the same stencils, yo
    the oracle's, ybound the bound on their difference."""
    sgn = sg.astype(np.float64)
    net = sgn * yo
    hf_valid = (shf >= 1) & (shf <= 3)

    def expected(flag):
        use_hf = flag & hf_valid
        return use_hf, np.where(flag, np.where(use_hf, shf, shf | 8), 8)

    flag = two | (np.abs(net) < kappa_lo)
    # an oracle output within the bound of the threshold may fall on either side on the GPU
    either = ~two & (np.abs(np.abs(net) - kappa_lo) <= ybound)
    hf_a, st_a = expected(flag)
    hf_b, st_b = expected(~flag)
    took_a = sc == st_a
    assert np.all(took_a | (either & (sc == st_b)))
    use_hf = np.where(took_a, hf_a, hf_b)
    assert np.all(np.abs(kc[use_hf] - khf[use_hf]) <= 1e-12)
    assert np.all(np.abs(kc[~use_hf] - net[~use_hf]) <= ybound[~use_hf])
    # the fused curvature kernel gives the forward kernel's outputs
    assert np.array_equal(kc[~use_hf], (sgn * y)[~use_hf])


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
    # the network on the oracle's stencils, with its records, bounds the GPU output
    y = torch.zeros(len(cells), dtype=torch.float32, device="cuda:0")
    acts = torch.zeros((len(cells), 768), dtype=torch.uint8, device="cuda:0")
    ctx.mlp_forward(_dev(P), _dev(xs), y, acts)
    torch.cuda.synchronize()
    assert nm == len(cells)
    kap, st = kap.cpu().numpy().ravel(), st.cpu().numpy().ravel()
    y = y.cpu().numpy().astype(np.float64)
    h1, h2 = _records(acts.cpu().numpy())
    _, _, yo, ybound = _forward_chain(P, xs, h1, h2, y)
    khf, shf = oracle.curvature_hf(c)
    khf, shf = khf.ravel(), shf.ravel()
    two = _two_interfaces(c, cells)
    _check_combined(kap[cells], st[cells], khf[cells], shf[cells], sg, y, yo, ybound, kappa_lo, two)
    other = np.setdiff1d(np.arange(c.size), cells)
    assert np.all(st[other] == 0) and np.all(np.isnan(kap[other]))
    if kappa_lo == 0.0:
        assert np.all(st[cells][~two] == 8)


def _two_interfaces(c, cells):
    nz, ny, nx = c.shape
    return np.array([oracle.two_interfaces(block_at(c, p // (nx * ny), (p // nx) % ny, p % nx)) for p in cells],
                    dtype=bool)


def test_curvature_mlp_two_interfaces(ctx):
    """27 copies of a block built to hold two interfaces (the oracle's hand-worked one, every value
    moved by up to 0.05) in a 24^3 field: with kappa_lo = 0 only the two-interface trigger
    sends cells to the height functions, and the GPU must flag exactly the oracle's cells."""
    import torch

    from test_oracle_two_interfaces import _hand_block

    rng = np.random.default_rng(71)
    c = np.zeros((24, 24, 24))
    for a in range(3):
        for b in range(3):
            for d in range(3):
                k, j, i = 4 + 7 * a, 4 + 7 * b, 4 + 7 * d
                c[k - 1:k + 2, j - 1:j + 2, i - 1:i + 2] = np.clip(
                    _hand_block() + rng.uniform(-0.05, 0.05, (3, 3, 3)), 0.0, 1.0)
    P = random_params(72, scale=0.3)
    cells, xs, sg = canonical_inputs(c)
    two = _two_interfaces(c, cells)
    assert two.sum() >= 20
    note(f"curvature mlp two interfaces: {len(cells)} cells, {int(two.sum())} flagged")
    kap = torch.zeros(c.shape, dtype=torch.float64, device="cuda:0")
    st = torch.zeros(c.shape, dtype=torch.uint8, device="cuda:0")
    nm = ctx.curvature_mlp(_dev(c), _dev(P), 0.0, kap, st)
    y = torch.zeros(len(cells), dtype=torch.float32, device="cuda:0")
    acts = torch.zeros((len(cells), 768), dtype=torch.uint8, device="cuda:0")
    ctx.mlp_forward(_dev(P), _dev(xs), y, acts)
    torch.cuda.synchronize()
    assert nm == len(cells)
    kap, st = kap.cpu().numpy().ravel(), st.cpu().numpy().ravel()
    y = y.cpu().numpy().astype(np.float64)
    h1, h2 = _records(acts.cpu().numpy())
    _, _, yo, ybound = _forward_chain(P, xs, h1, h2, y)
    khf, shf = oracle.curvature_hf(c)
    khf, shf = khf.ravel(), shf.ravel()
    _check_combined(kap[cells], st[cells], khf[cells], shf[cells], sg, y, yo, ybound, 0.0, two)
    assert np.all((st[cells] != 8) == two)


def test_curvature_mlp_full_size(ctx, drops512):
    """One 512^3 field of the benchmark workload with the trained weights, as
    the benchmark runs it: the count of mixed cells, and 4096 sampled mixed
    cells against the oracle's stencils, network and height functions."""
    import torch

    from paper_2407_07463_amd import training
    from mlp_fixtures import block_at

    P, meta = training.load_weights()
    c = drops512["c"][0]
    note("curvature mlp drops512 tracer 0 (full size)")
    cd = _dev(c)
    kap = torch.zeros(c.shape, dtype=torch.float64, device="cuda:0")
    st = torch.zeros(c.shape, dtype=torch.uint8, device="cuda:0")
    nm = ctx.curvature_mlp(cd, _dev(P), meta["kappa_lo"], kap, st)
    torch.cuda.synchronize()
    mixed = np.flatnonzero((c > 1e-12) & (c < 1.0 - 1e-12))  # interface cells
    assert nm == len(mixed)
    rng = np.random.default_rng(7)
    cells = np.sort(rng.choice(mixed, 4096, replace=False))
    nz, ny, nx = c.shape
    xs = np.zeros((len(cells), 27), dtype=np.float32)
    sg = np.zeros(len(cells), dtype=np.int8)
    for q, p in enumerate(cells):
        xs[q], sg[q] = oracle.canonical_stencil(block_at(c, p // (nx * ny), (p // nx) % ny, p % nx))
    y = torch.zeros(len(cells), dtype=torch.float32, device="cuda:0")
    acts = torch.zeros((len(cells), 768), dtype=torch.uint8, device="cuda:0")
    ctx.mlp_forward(_dev(P), _dev(xs), y, acts)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    h1, h2 = _records(acts.cpu().numpy())
    _, _, yo, ybound = _forward_chain(P, xs, h1, h2, y)
    khf, shf = oracle.curvature_hf(c)
    kc = kap.cpu().numpy().ravel()[cells]
    sc = st.cpu().numpy().ravel()[cells]
    _check_combined(kc, sc, khf.ravel()[cells], shf.ravel()[cells], sg, y, yo, ybound, meta["kappa_lo"],
                    _two_interfaces(c, cells))
