"""Pins for the learned-proposal oracle (oracle/learned.py): each function is
checked against something other than itself -- brute-force loops, closed
forms, library routines, finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import learned as ol


def _cn(g, n):
    return (g.normal(size=n) + 1j * g.normal(size=n)) / np.sqrt(2)


# ---------------------------------------------------------------- STFT map
def test_hann_is_the_periodic_library_window():
    assert np.allclose(ol.hann(), scipy.signal.get_window("hann", 256, fftbins=True), rtol=0, atol=1e-15)


def test_stft_power_brute_force_dft():
    g = np.random.default_rng(0)
    x = _cn(g, 700).astype(np.complex64)
    P = ol.stft_power(x)
    F = (700 - 256) // 128 + 1
    assert P.shape == (F, 256)
    w = ol.hann()
    for f in range(F):
        for b in (0, 1, 77, 128, 255):
            acc = 0j
            for n in range(256):
                acc += w[n] * complex(x[128 * f + n]) * np.exp(-2j * np.pi * b * n / 256)
            assert abs(P[f, b] - abs(acc) ** 2) <= 1e-10 * max(1.0, abs(acc) ** 2)


@pytest.mark.parametrize("b0", [0, 5, 128, 255])
def test_stft_tone_closed_form(b0):
    """A tone on bin b0: sum(w) = 128 in b0, 64 in each neighbour, 0 elsewhere."""
    n = np.arange(256 + 128 * 6)
    x = np.exp(2j * np.pi * b0 * n / 256)
    P = ol.stft_power(x)
    want = np.zeros(256)
    want[b0] = 128.0 ** 2
    want[(b0 + 1) % 256] = 64.0 ** 2
    want[(b0 - 1) % 256] = 64.0 ** 2
    assert np.allclose(P, want[None, :], rtol=0, atol=1e-8)


def test_stft_parseval():
    g = np.random.default_rng(1)
    x = _cn(g, 256 + 128 * 9)
    P = ol.stft_power(x)
    w = ol.hann()
    for f in range(P.shape[0]):
        e = np.sum(np.abs(w * x[128 * f:128 * f + 256]) ** 2)
        assert abs(P[f].sum() - 256 * e) <= 1e-10 * 256 * e


def test_num_frames_edges():
    assert ol.num_frames(255) == 0
    assert ol.num_frames(256) == 1
    assert ol.num_frames(383) == 1
    assert ol.num_frames(384) == 2
    assert ol.num_frames(1 << 20) == 8191


def test_lower_median():
    g = np.random.default_rng(2)
    v = g.random(1001)
    assert ol.lower_median(v) == np.median(v)
    v = g.random(1000)
    assert ol.lower_median(v) == np.partition(v, 499)[499]
    assert ol.lower_median([3.0, 1.0]) == 1.0


def test_power_map_gain_invariant_and_median_zero():
    g = np.random.default_rng(3)
    x = _cn(g, 256 + 128 * 40)
    m1, med1 = ol.power_map(x)
    m2, med2 = ol.power_map(7.5 * x)
    assert np.allclose(m1, m2, atol=1e-12)
    assert abs(med2 / med1 - 7.5 ** 2) < 1e-12
    assert ol.lower_median(m1) == pytest.approx(0.0, abs=1e-15)


def test_frame_labels_brute_force():
    n, L = 128 * 40 + 256, 1000
    delays = [0, 1700, 1790, 4500]
    lab = ol.frame_labels(n, delays, L)
    inside = np.zeros(n, bool)
    for D in delays:
        inside[D:min(D + L, n)] = True
    for f in range(ol.num_frames(n)):
        cnt = inside[128 * f:128 * f + 256].sum()
        assert lab[f] == (1.0 if cnt >= 128 else 0.0), f


# ---------------------------------------------------------------- network
def test_conv_same_brute_force():
    g = np.random.default_rng(4)
    F, cin, cout, d = 9, 3, 2, 2
    h = g.normal(size=(F, cin))
    W = g.normal(size=(5, cin, cout))
    b = g.normal(size=cout)
    out = ol.conv_same(h, W, b, d)
    for f in range(F):
        for o in range(cout):
            acc = b[o]
            for i in range(5):
                src = f + d * (i - 2)
                if 0 <= src < F:
                    for c in range(cin):
                        acc += W[i, c, o] * h[src, c]
            assert abs(out[f, o] - acc) < 1e-12


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_conv_same_is_library_correlation(d):
    """One channel: correlation with the dilated kernel, 'same' alignment."""
    g = np.random.default_rng(5 + d)
    F = 50
    h = g.normal(size=(F, 1))
    W = g.normal(size=(5, 1, 1))
    k = np.zeros(4 * d + 1)
    k[::d] = W[:, 0, 0]
    ref = scipy.signal.correlate(h[:, 0], k, mode="same", method="direct")
    assert np.allclose(ol.conv_same(h, W, np.zeros(1), d)[:, 0], ref, atol=1e-12)


def test_cnn_backward_finite_differences():
    g = np.random.default_rng(6)
    F, cin = 24, 6
    net = ol.init_cnn(7, cin=cin)
    for l in range(4):
        net.b[l] = g.normal(0, 0.1, size=64)
    net.bh = 0.3
    m = g.normal(size=(F, cin))
    dy = g.normal(size=F)
    y, h = ol.cnn_forward(net, m)
    grads = ol.cnn_backward(net, h, dy)
    params = net.params()
    eps = 1e-6
    for name, arr in params.items():
        flat = arr.reshape(-1)
        gflat = np.asarray(grads[name]).reshape(-1)
        scale = np.max(np.abs(gflat)) + 1e-30
        idx = g.choice(flat.size, size=min(flat.size, 40), replace=False)
        for i in idx:
            p = {k: v.copy() for k, v in params.items()}
            p[name].reshape(-1)[i] += eps
            yp = ol.cnn_forward(ol.CNN.from_params(p), m)[0] @ dy
            p[name].reshape(-1)[i] -= 2 * eps
            ym = ol.cnn_forward(ol.CNN.from_params(p), m)[0] @ dy
            fd = (yp - ym) / (2 * eps)
            assert abs(fd - gflat[i]) <= 1e-7 * scale + 1e-9 * abs(gflat[i]), (name, i, fd, gflat[i])


def test_bce_against_probability_form_and_gradient():
    g = np.random.default_rng(8)
    z = g.normal(0, 3, size=200)
    y = (g.random(200) < 0.3).astype(float)
    pw = 4.0
    loss, dz = ol.bce_with_logits(z, y, pw)
    s = 1.0 / (1.0 + np.exp(-z))
    direct = np.mean(-(pw * y * np.log(s) + (1 - y) * np.log(1 - s)))
    assert abs(loss - direct) < 1e-12
    eps = 1e-6
    for i in range(0, 200, 17):
        zp, zm = z.copy(), z.copy()
        zp[i] += eps
        zm[i] -= eps
        fd = (ol.bce_with_logits(zp, y, pw)[0] - ol.bce_with_logits(zm, y, pw)[0]) / (2 * eps)
        assert abs(fd - dz[i]) < 1e-8


def test_adam_first_step_closed_form():
    """t = 1: the bias-corrected moments are g and g^2, so p -= lr g / (|g| + eps)."""
    g = np.random.default_rng(9)
    p = g.normal(size=100)
    grad = g.normal(size=100)
    p0 = p.copy()
    m, v = np.zeros(100), np.zeros(100)
    ol.adam_step(p, grad, m, v, 1, lr=1e-2)
    assert np.allclose(p, p0 - 1e-2 * grad / (np.abs(grad) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)


def test_adam_constant_gradient_moves_lr_per_step():
    """A constant gradient keeps m_hat = g and v_hat = g^2 at every t."""
    p = np.array([1.0, -2.0])
    grad = np.array([0.5, -3.0])
    m, v = np.zeros(2), np.zeros(2)
    for t in range(1, 6):
        ol.adam_step(p, grad, m, v, t, lr=0.1)
    assert np.allclose(p, [1.0 - 0.5, -2.0 + 0.5], atol=1e-7)


# ---------------------------------------------------------------- proposals
def test_window_scores_are_a_library_convolution():
    g = np.random.default_rng(10)
    y = g.normal(size=500)
    c = ol.window_scores(y)
    ref = np.convolve(y, np.ones(128), mode="full")[64:64 + 500]
    assert np.allclose(c, ref, atol=1e-10)


def test_propose_threshold():
    c = np.array([0.0, 5.0, 9.0, 1.0, 9.0, -3.0])
    assert ol.propose(c, 2.0).tolist() == [1, 2, 4]
    assert ol.propose(c, 9.0).tolist() == [2, 4]
    assert ol.propose(c, 100.0).tolist() == []


def test_a_transmission_is_proposed_by_any_frame_it_covers():
    """The proposed ranges of every frame lying wholly inside a replica at lag tau
    contain tau, and no other frame's range does."""
    n, L = 1 << 16, 16384
    for tau in (0, 1, 127, 128, 30000, n - L):
        inside = [f for f in range(ol.num_frames(n)) if 128 * f >= tau and 128 * f + 256 <= tau + L]
        for f in range(ol.num_frames(n)):
            r = ol.frame_lag_range(f, n, L)
            hit = r is not None and r[0] <= tau <= r[1]
            assert hit == (f in inside), (tau, f)


def test_frame_lag_range_brute_force():
    n, L = 5000, 1000
    for f in range(ol.num_frames(n)):
        want = [t for t in range(n - L + 1) if t <= 128 * f and t + L >= 128 * f + 256]
        r = ol.frame_lag_range(f, n, L)
        if not want:
            assert r is None
        else:
            assert r == (want[0], want[-1]) and len(want) == want[-1] - want[0] + 1


def test_segments_for_ranges_brute_force():
    n, L, V = 20000, 1000, 777
    lags = n - L + 1
    ranges = [(0, 5), (776, 777), (5000, 6200), (lags - 3, lags - 1), None]
    segs = ol.segments_for_ranges(ranges, V, n, L)
    want = sorted({t // V for r in ranges if r for t in range(r[0], r[1] + 1)})
    assert segs.tolist() == want



def test_power_map_of_an_empty_block_is_zero():
    m, med = ol.power_map(np.zeros(256 + 128 * 3, np.complex64))
    assert med == 0.0 and m.shape == (4, 256) and not m.any()


def test_bf16_round_is_the_library_conversion():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(12)
    v = np.concatenate([g.normal(0, 10, 5000), g.normal(0, 1e-30, 100), [0.0, -0.0, 1.0, 3.0, 65504.0]])
    # values exactly halfway between two bf16 numbers: ties go to the even significand
    base = np.array([1.0, 1.0078125, 3.0, -5.5], dtype=np.float32).view(np.uint32)
    ties = (base + 0x8000).view(np.float32).astype(np.float64)
    v = np.concatenate([v, ties]).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ol.bf16_round(v), want)


def test_bf16_forward_rounds_every_layer_output():
    g = np.random.default_rng(13)
    net = ol.init_cnn(14, cin=8)
    m = g.normal(size=(30, 8))
    y, h = ol.cnn_forward(ol.bf16_network(net), m, act_round=ol.bf16_round)
    for a in h[1:]:
        assert np.array_equal(a, ol.bf16_round(a))
    y64, _ = ol.cnn_forward(net, m)
    assert 0 < np.linalg.norm(y - y64) / np.linalg.norm(y64) < 0.05
