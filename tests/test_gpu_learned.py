"""Proposal stage on the GPU against the FP64 oracle (oracle/learned.py):
power map, network forward / gradients / Adam (FP32 reference arithmetic to
1e-5, bf16 MFMA within 2e-2 relative L2 per tensor), the synthetic generator,
and the proposal search (a bit-exact subset of the exhaustive search)."""
import numpy as np
import pytest

import oracle
import siggen
from oracle import learned as ol

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS = 8e6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _net(prec, cin=256, max_rows=1 << 14, max_block_len=None):
    from paper_2005_10445_amd.proposals import Network
    if max_block_len is None:                       # the longest block whose frames fit
        max_block_len = min(1 << 20, (max_rows - 1) * 128 + 256)
    return Network(prec, in_channels=cin, max_rows=max_rows, max_block_len=max_block_len)


def _flat(net_o: "ol.CNN") -> np.ndarray:
    parts = []
    for l in range(4):
        parts += [net_o.W[l].reshape(-1), net_o.b[l]]
    parts += [net_o.wh, np.array([net_o.bh])]
    return np.concatenate(parts).astype(np.float64)


def _grads_flat(g) -> np.ndarray:
    parts = []
    for l in range(4):
        parts += [np.asarray(g[f"W{l}"]).reshape(-1), np.asarray(g[f"b{l}"])]
    parts += [np.asarray(g["wh"]), np.asarray(g["bh"]).reshape(-1)]
    return np.concatenate(parts)


def _segments(net_o, cin):
    """(name, slice) of each parameter tensor in the flat vector."""
    out, off = [], 0
    for l in range(4):
        c = cin if l == 0 else 64
        out.append((f"W{l}", slice(off, off + 5 * c * 64)))
        off += 5 * c * 64
        out.append((f"b{l}", slice(off, off + 64)))
        off += 64
    out.append(("wh", slice(off, off + 64)))
    out.append(("bh", slice(off + 64, off + 65)))
    return out


def _oracle_batch(net_o, inp, nblocks, labels, pw, act_round=None):
    """Logits, mean loss and flat gradient of a batch of equal blocks."""
    F = inp.shape[0] // nblocks
    ys, hs = [], []
    for b in range(nblocks):
        y, h = ol.cnn_forward(net_o, inp[b * F:(b + 1) * F], act_round)
        ys.append(y)
        hs.append(h)
    y = np.concatenate(ys)
    loss, dz = ol.bce_with_logits(y, labels, pw)
    g = None
    for b in range(nblocks):
        gb = _grads_flat(ol.cnn_backward(net_o, hs[b], dz[b * F:(b + 1) * F]))
        g = gb if g is None else g + gb
    return y, loss, g


def _rand_net(seed, cin):
    g = np.random.default_rng(seed)
    net_o = ol.init_cnn(seed, cin=cin)
    for l in range(4):
        net_o.b[l] = g.normal(0, 0.05, size=64)
    net_o.bh = -0.5
    return net_o


def _bf16(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to bf16 (nearest even) and back, as the device stores them."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- power map
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_power_map_against_oracle(dev, prec):
    T, C, spc = 4, 512, 2
    chips = siggen.make_codes(900, T, C)
    freqs, _ = oracle.snap_bins(FS, C * spc, 3, 0.0, 20e3)
    n = 256 + 128 * 300 + 77
    x, _ = siggen.make_block(901, n, chips, spc, FS, freqs, 3, snr_db=(0.0, 10.0))
    with _net(prec) as net:
        m, med = net.power_map(torch.from_numpy(x).to(dev))
        m = m.float().cpu().numpy().astype(np.float64)
    ref, med_ref = ol.power_map(x)
    assert m.shape == ref.shape == (ol.num_frames(n), 256)
    assert abs(med - med_ref) <= 1e-5 * med_ref
    P = ol.stft_power(x)
    ok = P > 1e-4 * med_ref
    tol = 1e-3 if prec == "fp32" else 1e-3 + 2.0 ** -8 * np.abs(ref)
    err = np.abs(m - ref)
    assert np.all((err <= tol)[ok]), float(np.max(err[ok]))
    assert np.all(m[~ok] < np.log(2e-4))


def test_power_map_tone_and_empty_block(dev):
    n = 256 + 128 * 20
    b0 = 37
    x = np.exp(2j * np.pi * b0 * np.arange(n) / 256).astype(np.complex64)
    with _net("fp32") as net:
        m, med = net.power_map(torch.from_numpy(x).to(dev))
        m = m.cpu().numpy()
        z, medz = net.power_map(torch.zeros(n, dtype=torch.complex64, device=dev))
    # 3 of 256 bins hold power: the lower median is a leakage-floor value, tiny
    assert med < 1e-6 and np.argmax(m[5]) == b0
    assert medz == 0.0 and not z.cpu().numpy().any()


# ---------------------------------------------------------------- network
@pytest.mark.parametrize("nblocks,F,cin", [(1, 37, 48), (2, 70, 64)])
def test_forward_gradients_fp32_against_oracle(dev, nblocks, F, cin):
    g = np.random.default_rng(10 + F)
    net_o = _rand_net(20 + F, cin)
    inp = g.normal(size=(nblocks * F, cin))
    labels = (g.random(nblocks * F) < 0.3).astype(np.float64)
    pw = 3.0
    y_ref, loss_ref, g_ref = _oracle_batch(net_o, inp, nblocks, labels, pw)
    with _net("fp32", cin=cin, max_rows=4096) as net:
        net.set_params(_flat(net_o))
        ti = torch.from_numpy(inp.astype(np.float32)).to(dev)
        tl = torch.from_numpy(labels.astype(np.float32)).to(dev)
        y = net.forward(ti, nblocks).cpu().numpy()
        loss, grad = net.gradients(ti, tl, pw, nblocks)
        grad = grad.cpu().numpy()
    assert np.max(np.abs(y - y_ref)) <= 1e-5 * (1 + np.max(np.abs(y_ref)))
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    for name, sl in _segments(net_o, cin):
        a, b = grad[sl], g_ref[sl]
        assert np.max(np.abs(a - b)) <= 1e-5 * (np.max(np.abs(b)) + 1e-12), name


# (2, 150): pieces of 64 rows with and without a block start near them; (8, 20):
# a block start in every piece, most pairs of the outer taps cross one; (1, 600):
# mostly pieces with no block start near them, for every dilation
@pytest.mark.parametrize("nblocks,F", [(2, 150), (8, 20), (1, 600)])
def test_forward_gradients_bf16_against_oracle(dev, nblocks, F):
    g = np.random.default_rng(3 + F)
    cin = 256
    net_o = _rand_net(4, cin)
    inp = _bf16(g.normal(size=(nblocks * F, cin)))
    labels = (g.random(nblocks * F) < 0.3).astype(np.float64)
    pw = 2.0
    # reference: FP64 gradient of the bf16 network (weights and layer outputs in bf16)
    y_ref, loss_ref, g_ref = _oracle_batch(ol.bf16_network(net_o), inp, nblocks, labels, pw, ol.bf16_round)
    with _net("bf16", cin=cin, max_rows=4096) as net:
        net.set_params(_flat(net_o))
        ti = torch.from_numpy(inp.astype(np.float32)).to(dev).to(torch.bfloat16)
        tl = torch.from_numpy(labels.astype(np.float32)).to(dev)
        y = net.forward(ti, nblocks).cpu().numpy()
        loss, grad = net.gradients(ti, tl, pw, nblocks)
        grad = grad.cpu().numpy()
        _, grad2 = net.gradients(ti, tl, pw, nblocks)
        grad2 = grad2.cpu().numpy()
    # the conv layers' gradients are summed in a fixed order: the same batch
    # gives them bit for bit (the head's sums use atomics)
    for name, sl in _segments(net_o, cin):
        if name[0] in "Wb" and name[1:].isdigit():
            assert np.array_equal(grad[sl], grad2[sl]), name

    def rel(a, b):
        return np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)

    assert rel(y, y_ref) <= 2e-2
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref
    for name, sl in _segments(net_o, cin):
        assert rel(grad[sl], g_ref[sl]) <= 2e-2, (name, rel(grad[sl], g_ref[sl]))
        if name.startswith("W"):
            # each tap on its own: a tap whose rows cross a block start is a small part of its layer
            a, b = grad[sl].reshape(5, -1), g_ref[sl].reshape(5, -1)
            for i in range(5):
                assert rel(a[i], b[i]) <= 3e-2, (name, i, rel(a[i], b[i]))


def _unflat(p, cin) -> "ol.CNN":
    W, b, off = [], [], 0
    for l in range(4):
        c = cin if l == 0 else 64
        W.append(p[off:off + 5 * c * 64].reshape(5, c, 64).copy())
        off += 5 * c * 64
        b.append(p[off:off + 64].copy())
        off += 64
    return ol.CNN(W, b, p[off:off + 64].copy(), float(p[off + 64]))


def test_adam_steps_against_oracle(dev):
    """The optimiser on its own: the oracle's Adam applied to the gradient the
    device computed (gradient parity is tested above; Adam's first steps move
    every weight by about lr * sign(g), so FP32-vs-FP64 noise in a near-zero
    gradient would otherwise dominate the comparison)."""
    g = np.random.default_rng(5)
    F, cin = 50, 16
    p = _flat(_rand_net(6, cin)).astype(np.float32).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    lr = 1e-2
    with _net("fp32", cin=cin, max_rows=1024) as net:
        net.set_params(p)
        for t in (1, 2, 3):
            inp = g.normal(size=(F, cin))
            labels = (g.random(F) < 0.4).astype(np.float64)
            ti = torch.from_numpy(inp.astype(np.float32)).to(dev)
            tl = torch.from_numpy(labels.astype(np.float32)).to(dev)
            _, grad = net.gradients(ti, tl, 2.0)
            net.adam_step(lr)
            ol.adam_step(p, grad.cpu().numpy().astype(np.float64), m, v, t, lr=lr)
            got = net.get_params().astype(np.float64)
            assert np.max(np.abs(got - p)) <= 1e-6 * lr + 1e-6 * np.max(np.abs(p)), t
            p = got.copy()                     # continue from the device's FP32 state


# ---------------------------------------------------------------- generator
def test_synthetic_generator_statistics(dev):
    from paper_2005_10445_amd.proposals import SynthTransmission
    n, C, spc = 1 << 18, 8192, 2
    L = C * spc
    with _net("bf16") as net:
        x0 = net.synth_block(7, 0, n, C, spc, []).cpu().numpy()
        tx = SynthTransmission(delay=100000, freq_over_fs=1.0 / 64, amp=3.0, phase0=0.25, code=5)
        x1 = net.synth_block(7, 0, n, C, spc, [tx]).cpu().numpy()
        x2 = net.synth_block(7, 1, n, C, spc, []).cpu().numpy()
    p0 = np.abs(x0) ** 2
    assert abs(p0.mean() - 1.0) < 0.01
    assert abs(np.var(x0.real) - 0.5) < 0.01 and abs(np.var(x0.imag) - 0.5) < 0.01
    assert abs(np.mean(x0.real * x0.imag)) < 0.01
    assert np.corrcoef(np.abs(x0[:4096]), np.abs(x2[:4096]))[0, 1] < 0.05   # other block, other noise
    d = x1 - x0                                                               # the transmission alone
    assert np.all(np.abs(d[:100000]) < 1e-5) and np.all(np.abs(d[100000 + L:]) < 1e-5)
    s = d[100000:100000 + L] * np.exp(-2j * np.pi * (np.arange(100000, 100000 + L) / 64 + 0.25))
    assert np.allclose(np.abs(s.real), 3.0, atol=1e-3) and np.max(np.abs(s.imag)) < 1e-3
    chips = np.sign(s.real[::2])
    assert np.all(s.real[1::2] * chips > 0)                 # held for spc samples
    assert abs(chips.mean()) < 0.05                         # balanced +/-1


def test_training_labels_match_the_oracle(dev):
    """Frame labels of generated batches, bit for bit against the oracle and a
    brute-force count: overlapping transmissions (a union, not a sum), one cut
    by the block's end, frames exactly half covered, a block without
    transmissions, and a template shorter than a frame."""
    from paper_2005_10445_amd.proposals import SynthTransmission
    g = np.random.default_rng(12)
    n = 1 << 16
    for C, spc in ((8192, 2), (50, 2)):
        L = C * spc
        delays = [
            [0, 5000, 5100, n - L // 2],                       # block start, an overlap, the end
            [],
            [int(d) for d in g.integers(0, n, 20)],            # many, overlapping
            [128 * 40 + 128, 128 * 90 - 1, 128 * 300 + 127],   # boundaries of half-covered frames
        ]
        txs = [[SynthTransmission(delay=d, freq_over_fs=0.0, amp=1.0, phase0=0.0, code=i) for i, d in enumerate(b)]
               for b in delays]
        with _net("bf16", max_rows=1 << 12) as net:
            got = net.synth_labels(3, 0, n, C, spc, txs).cpu().numpy().reshape(len(txs), -1)
        for b, ds in enumerate(delays):
            want = ol.frame_labels(n, ds, L)
            cover = np.zeros(n, dtype=bool)
            for d in ds:
                cover[d:min(d + L, n)] = True
            brute = np.array([cover[128 * f:128 * f + 256].sum() >= 128 for f in range(want.size)], dtype=np.float64)
            assert np.array_equal(want, brute), (C, b)
            assert np.array_equal(got[b].astype(np.float64), want), (C, b)
            if ds and L >= 256:
                assert 0 < want.sum() < want.size, (C, b)


def test_training_reduces_loss(dev):
    from paper_2005_10445_amd.proposals import SynthTransmission
    g = np.random.default_rng(8)
    n, C, spc = 1 << 17, 8192, 2
    L = C * spc
    net_o = ol.init_cnn(9)
    losses = []
    with _net("bf16", max_rows=1 << 12) as net:
        net.set_params(_flat(net_o))
        for step in range(40):
            txs = []
            for b in range(2):
                lst = []
                for i in range(3):
                    lst.append(SynthTransmission(int(g.integers(0, n - L)), float(g.integers(-5, 6)) * 976.5625 / FS,
                                                 float(10 ** (g.uniform(-3, 3) / 20)), float(g.random()),
                                                 int(g.integers(0, 2 ** 31))))
                txs.append(lst)
            losses.append(net.train_synthetic(11, 2 * step, n, C, spc, txs, pos_weight=2.0, lr=3e-3))
    assert all(np.isfinite(losses))
    assert np.mean(losses[-5:]) < 0.7 * np.mean(losses[:5]), losses


# ---------------------------------------------------------------- proposal search
def _learned_setup(dev, seed=30):
    from paper_2005_10445_amd import Plan
    T, C, spc, K, step = 8, 2048, 2, 3, 5e3
    L = C * spc
    n = 1 << 18
    chips = siggen.make_codes(seed, T, C)
    plan = Plan(chips, spc, FS, num_bins=K, bin_step_hz=step, max_block_len=n, fft_len=8192)
    x, txs = siggen.make_block(seed + 1, n, chips, spc, FS, plan.freqs_hz, 4, snr_db=(-5.0, 5.0))
    return plan, chips, x, txs, L


def test_proposal_search_is_a_bit_exact_subset(dev):
    plan, chips, x, txs, L = _learned_setup(dev)
    from paper_2005_10445_amd.proposals import LearnedParams
    n = x.size
    xt = torch.from_numpy(x).to(dev)
    V = plan.geometry["valid_per_segment"]
    net_o = _rand_net(31, 256)
    with plan, _net("bf16", max_block_len=n) as net:
        net.set_params(_flat(net_o))
        full = {d.tag: d for d in plan.detect(xt)}
        m, _ = net.power_map(xt)
        y = net.forward(m).cpu().numpy().astype(np.float64)
        # a threshold that proposes some frames but not all: the 97th percentile score
        c64 = ol.window_scores(y)
        kappa = float(np.float32(np.quantile(c64, 0.97)))
        lp = LearnedParams(kappa=kappa, max_fraction=1.0, floor_db=0.0)
        dets, rep = net.detect(plan, xt, lp)
    # window scores summed in FP32 in the device's order, so that candidate
    # decisions (which compare nearly equal sums) are taken on the same values
    y32 = y.astype(np.float32)
    F = y32.size
    c = np.zeros(F)
    for f in range(F):
        acc = np.float32(0.0)
        for i in range(max(0, f - 63), min(F, f + 65)):
            acc = np.float32(acc + y32[i])
        c[f] = float(acc)
    frames = ol.propose(c, kappa)
    segs = set(ol.segments_for_ranges([ol.frame_lag_range(int(f), n, L) for f in frames], V, n, L).tolist())
    assert rep.fallback == 0 and rep.proposals == len(frames)
    assert rep.segments == len(segs) and 0 < rep.segments < rep.total_segments
    got = {d.tag: d for d in dets}
    for t, d in got.items():                     # every proposal detection lies in a searched segment ...
        assert d.lag // V in segs
    for t, d in full.items():                    # ... and equals the exhaustive one when that peak is searched
        if d.lag // V in segs:
            e = got.get(t)
            assert e is not None and (e.bin, e.lag, e.toa, e.peak_power, e.z, e.energy) == \
                (d.bin, d.lag, d.toa, d.peak_power, d.z, d.energy), t


def test_proposal_search_fallbacks_equal_exhaustive(dev):
    plan, chips, x, txs, L = _learned_setup(dev, seed=40)
    from paper_2005_10445_amd.proposals import LearnedParams
    xt = torch.from_numpy(x).to(dev)
    with plan, _net("bf16", max_block_len=x.size) as net:
        net.set_params(_flat(_rand_net(41, 256)))
        key = lambda ds: [(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in ds]   # noqa: E731
        full = key(plan.detect(xt))
        dets, rep = net.detect(plan, xt, LearnedParams(kappa=-1e30, max_fraction=0.0, floor_db=0))
        assert rep.fallback == 1 and rep.segments == rep.total_segments and key(dets) == full
        # the noise floor: set by the first call; a 6 dB louder block falls back
        dets, rep = net.detect(plan, xt, LearnedParams(kappa=1e30, max_fraction=1.0, floor_db=1.0))
        assert rep.fallback == 0 and rep.segments == 0 and dets == []
        dets, rep = net.detect(plan, 2 * xt, LearnedParams(kappa=1e30, max_fraction=1.0, floor_db=1.0))
        assert rep.fallback == 2 and abs(rep.median / rep.floor - 4.0) < 0.5
        assert key(dets) == key(plan.detect(2 * xt))


def test_batched_proposal_search_equals_per_block(dev):
    """One batched search over the proposed segments of several blocks returns
    what per-block proposal searches return (floor updates in the same order),
    including a fallback block and a block shorter than a template."""
    from paper_2005_10445_amd import Plan
    from paper_2005_10445_amd.proposals import LearnedParams
    T, C, spc, K, step = 8, 2048, 2, 3, 5e3
    L = C * spc
    chips = siggen.make_codes(50, T, C)
    lens = [1 << 18, 150000, L - 5, 200001]
    net_params = _flat(_rand_net(51, 256))
    with Plan(chips, spc, FS, num_bins=K, bin_step_hz=step, max_block_len=1 << 18, fft_len=8192,
              max_batch_blocks=4) as plan:
        xs = []
        for b, n in enumerate(lens):
            ntx = 3 if n > L else 0
            x, _ = siggen.make_block(52 + b, n, chips, spc, FS, plan.freqs_hz, ntx, snr_db=(-5.0, 5.0))
            xs.append(torch.from_numpy(x).to(dev))
        xs[3] = 1.5 * xs[3]                        # 3.5 dB louder: the floor rule fires
        with _net("bf16", max_block_len=1 << 18) as net:
            net.set_params(net_params)
            m, _ = net.power_map(xs[0])
            c = ol.window_scores(net.forward(m).cpu().numpy().astype(np.float64))
            lp = LearnedParams(kappa=float(np.quantile(c, 0.9)), max_fraction=0.6, floor_db=1.0)
            per, per_rep = [], []
            for b, x in enumerate(xs):
                dets, rep = net.detect(plan, x, lp)
                for d in dets:
                    d.block = b
                per += dets
                per_rep.append(rep)
        with _net("bf16", max_block_len=1 << 18) as net:
            net.set_params(net_params)
            batch, reps = net.detect_batch(plan, xs, lp)
    key = lambda ds: [(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z) for d in ds]   # noqa: E731
    assert key(batch) == key(per)
    assert [(r.proposals, r.segments, r.total_segments, r.fallback) for r in reps] == \
        [(r.proposals, r.segments, r.total_segments, r.fallback) for r in per_rep]
    assert reps[2].total_segments == 0 and reps[3].fallback == 2
