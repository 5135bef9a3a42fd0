"""Tracking-mode tasks (acq_track_batch): each task searches one block for one
tag.  Against the FP64 oracle's tracking task, against the searching path
restricted to the same tag, with graph replay, and at the tracking workload's
full size."""
import numpy as np
import pytest

import oracle
import siggen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS = 8e6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(dets, tasks, chips, spc, freqs, theta=None, method="direct"):
    L = chips.shape[1] * spc
    got = {d.block: d for d in dets}
    assert [d.block for d in dets] == sorted(got)              # task order
    for i, (x, tag) in enumerate(tasks):
        r = oracle.track(x, chips, spc, freqs, FS, tag, theta=theta, method=method)
        if r is None or not r["detected"]:
            assert i not in got or (r is not None and r["near_threshold"]), i
            continue
        if r["near_threshold"] and i not in got:
            continue
        d = got[i]
        assert d.tag == tag
        if not r["near_tie"]:
            assert (d.bin, d.lag) == (r["bin"], r["lag"]), (i, d, r)
        assert abs(d.toa - r["toa"]) <= 1e-3
        floor = max(r["peak_power"], L * r["block_power"])
        assert abs(d.peak_power - r["peak_power"]) <= 1e-9 * floor
        assert abs(d.z - r["z"]) <= 1e-9 * max(r["z"], 1.0)
        assert d.freq_hz == r["freq_hz"]


def _plan(chips, spc, K, N, M=0, **kw):
    from paper_2005_10445_amd import Plan
    return Plan(chips, spc, FS, num_bins=K, bin_step_hz=1000.0, max_block_len=N, fft_len=M, **kw)


def test_mixed_tasks_match_the_oracle(dev):
    """Uneven blocks (shorter than a template, exactly one template, 1.5
    templates, several segments), tasks sharing a block, repeated tags."""
    T, C, spc, K, M = 5, 300, 2, 5, 2048
    L = C * spc
    chips = siggen.make_codes(700, T, C)
    freqs = oracle.snap_bins(FS, L, K, 0.0, 1000.0)[0]
    blocks = []
    for i, (n, tags) in enumerate([(L - 1, []), (L, [1]), (3 * L // 2, [2]), (3 * L // 2, [0, 4]),
                                   (5000, [3, 1, 2]), (3 * L // 2, [])]):
        x, _ = siggen.make_block(701 + i, n, chips, spc, FS, freqs, len(tags), snr_db=(-3.0, 3.0), tags=tags,
                                 fracs=[0.0] * len(tags))
        blocks.append(x)
    tasks = [(blocks[0], 0), (blocks[1], 1), (blocks[1], 2), (blocks[2], 2), (blocks[3], 4), (blocks[3], 0),
             (blocks[3], 3), (blocks[4], 3), (blocks[4], 1), (blocks[4], 2), (blocks[4], 0), (blocks[5], 4),
             (blocks[2], 2)]
    dev_blocks = [torch.from_numpy(b).to(dev) for b in blocks]
    index = {id(b): j for j, b in enumerate(blocks)}
    with _plan(chips, spc, K, 5000, M, max_batch_blocks=len(tasks)) as plan:
        assert np.array_equal(plan.freqs_hz, freqs)
        dets = plan.track([(dev_blocks[index[id(x)]], t) for x, t in tasks])
    assert len(dets) >= 7
    _check(dets, tasks, chips, spc, freqs)


def test_tracking_equals_the_search_for_that_tag(dev):
    """With one explicit threshold, a tracking task returns exactly what the
    searching path returns for the same tag (same kernels, same FP64 values)."""
    T, C, spc, K, N = 6, 400, 2, 3, 9000
    chips = siggen.make_codes(710, T, C)
    L = C * spc
    freqs = oracle.snap_bins(FS, L, K, 0.0, 1000.0)[0]
    x, txs = siggen.make_block(711, N, chips, spc, FS, freqs, 4, snr_db=(-6.0, 0.0))
    xt = torch.from_numpy(x).to(dev)
    theta = 12.0
    with _plan(chips, spc, K, N, threshold=theta, max_batch_blocks=T) as plan:
        search = {d.tag: d for d in plan.detect(xt)}
        tracked = plan.track([(xt, t) for t in range(T)])
    assert {d.tag for d in tracked} == set(search)
    for d in tracked:
        s = search[d.tag]
        assert (d.bin, d.lag, d.toa, d.peak_power, d.z, d.energy, d.flags) == \
               (s.bin, s.lag, s.toa, s.peak_power, s.z, s.energy, s.flags)
    _check(tracked, [(x, t) for t in range(T)], chips, spc, freqs, theta=theta)


def test_graph_replay_and_interleaving(dev):
    """A captured tracking graph replayed on batches of different sizes, with
    searching batches (their own graph) and eager calls in between."""
    T, C, spc, K, M = 4, 256, 2, 3, 2048
    L = C * spc
    chips = siggen.make_codes(720, T, C)
    freqs = oracle.snap_bins(FS, L, K, 0.0, 1000.0)[0]
    batch = siggen.make_tracking_batch(721, chips, spc, FS, freqs, 12, snr_db=(-3.0, 3.0))
    tasks = [(torch.from_numpy(x).to(dev), t) for x, t, _ in batch]
    n = batch[0][0].size
    kw = dict(max_batch_blocks=12, max_batch_samples=12 * n)
    with _plan(chips, spc, K, n, M, **kw) as eager, _plan(chips, spc, K, n, M, graph=True, **kw) as graphed:
        want = eager.track(tasks)
        for sub in (tasks, tasks[:5], tasks[3:4], tasks):
            got = graphed.track(sub)
            ref = eager.track(sub)
            assert [(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in got] == \
                   [(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in ref]
            s1 = graphed.detect_batch([b for b, _ in sub])
            s2 = eager.detect_batch([b for b, _ in sub])
            assert [(d.block, d.tag, d.lag, d.peak_power) for d in s1] == \
                   [(d.block, d.tag, d.lag, d.peak_power) for d in s2]
    _check(want, [(x, t) for x, t, _ in batch], chips, spc, freqs)


def test_errors(dev):
    from paper_2005_10445_amd import AcqError
    chips = siggen.make_codes(730, 3, 100)
    x = torch.zeros(600, dtype=torch.complex64, device=dev)
    with _plan(chips, 2, 1, 600, max_batch_blocks=2) as plan:
        with pytest.raises(AcqError) as e:
            plan.track([(x, 3)])
        assert e.value.status == -1
        with pytest.raises(AcqError) as e:
            plan.track([(x, 0)] * 3)
        assert e.value.status == -1
        assert plan.track([(x, 0), (x, 2)]) == []          # all-zero block: z = 0
    with _plan(chips, 2, 1, 600, max_batch_blocks=2, max_batch_samples=700) as plan:
        with pytest.raises(AcqError) as e:
            plan.track([(x, 0), (x, 1)])
        assert e.value.status == -5


def test_tracking_workload_full_size(dev):
    """256 tasks of the tracking workload (256-tag bank, 21 bins, blocks of 1.5
    templates): every task whose packet is present at -15..-5 dB is found at its
    delay and bin; sampled tasks match the oracle (FFT-identity argmax, direct
    FP64 values)."""
    w = siggen.workload("tracking")
    chips = siggen.make_codes(w["seeds"][0], w["num_tags"], w["num_chips"])
    spc, K = w["spc"], w["num_bins"]
    L = chips.shape[1] * spc
    freqs = oracle.snap_bins(FS, L, K, w["bin_center_hz"], w["bin_step_hz"])[0]
    batch = siggen.make_tracking_batch(w["seeds"][0] + 1, chips, spc, FS, freqs, w["num_tasks"],
                                       block_factor=w["block_factor"], p_present=w["p_present"],
                                       n_other=w["n_other"], snr_db=w["snr_db"])
    n = batch[0][0].size
    tasks = [(torch.from_numpy(x).to(dev), t) for x, t, _ in batch]
    with _plan(chips, spc, K, n, max_batch_blocks=len(tasks), max_batch_samples=len(tasks) * n) as plan:
        dets = plan.track(tasks)
    got = {d.block: d for d in dets}
    present = [i for i, (_, t, txs) in enumerate(batch) if any(q.tag == t for q in txs)]
    assert len(present) > 200
    for i in present:
        tx = next(q for q in batch[i][2] if q.tag == batch[i][1])
        d = got[i]
        assert d.bin == tx.bin and abs(d.toa - (tx.delay + tx.frac)) <= 0.5
    sample = present[::32] + [i for i in range(len(batch)) if i not in present][:4]
    for i in sample:
        x, tag, _ = batch[i]
        r = oracle.track(x, chips, spc, freqs, FS, tag, method="fft")
        if not r["detected"]:
            assert i not in got or r["near_threshold"]
            continue
        d = got[i]
        if not r["near_tie"]:
            assert (d.bin, d.lag) == (r["bin"], r["lag"])
        assert abs(d.toa - r["toa"]) <= 1e-3
        assert abs(d.peak_power - r["peak_power"]) <= 1e-9 * max(r["peak_power"], L * r["block_power"])


def test_bins_per_item_do_not_change_results(dev):
    """Tracking work items over 1, 2, 3, K bins (and the per-launch choice) give
    identical detections: the peak key is an exact maximum."""
    T, C, spc, K, M = 6, 300, 2, 7, 2048
    L = C * spc
    chips = siggen.make_codes(740, T, C)
    freqs = oracle.snap_bins(FS, L, K, 0.0, 1000.0)[0]
    batch = siggen.make_tracking_batch(741, chips, spc, FS, freqs, 24, block_factor=2.5, snr_db=(-6.0, 0.0))
    tasks = [(torch.from_numpy(x).to(dev), t) for x, t, _ in batch]
    n = batch[0][0].size
    with _plan(chips, spc, K, n, M, max_batch_blocks=len(tasks)) as plan:
        runs = []
        for bins in (1, 2, 3, K, 0):
            tu = plan.tuning
            plan.set_tuning(tu["engine"], tu["tag_tile"], track_bins=bins)
            assert plan.tuning["track_bins"] == bins
            runs.append(plan.track(tasks))
    rows = [[(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z) for d in r] for r in runs]
    assert all(r == rows[0] for r in rows[1:])
    assert len(rows[0]) >= 15
    _check(runs[0], [(x, t) for x, t, _ in batch], chips, spc, freqs)
