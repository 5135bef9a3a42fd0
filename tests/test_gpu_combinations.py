"""Features used together: exact-frequency bins with 16-bit storage, batches,
graph replay, tracking tasks and the proposal search.  Each combination is
checked against the separately tested single-feature path and the FP64
oracle."""
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


def _plan(chips, spc, K, centre, step, nmax, M, **kw):
    from paper_2005_10445_amd import Plan
    return Plan(chips, spc, FS, num_bins=K, bin_center_hz=centre, bin_step_hz=step, max_block_len=nmax, fft_len=M,
                **kw)


def _setup(seed, T=6, C=300, spc=2, K=5, centre=321.0, step=7777.7, lens=(15037, 9000, 601, 20000)):
    chips = siggen.make_codes(seed, T, C)
    freqs = centre + (np.arange(K) - (K - 1) / 2) * step
    L = C * spc
    blocks = []
    for b, n in enumerate(lens):
        ntx = 2 if n > L + 10 else 0
        x, txs = siggen.make_block(seed + 1, n, chips, spc, FS, freqs, ntx, snr_db=(-3.0, 3.0), sub=b)
        blocks.append((x, txs))
    return chips, freqs, blocks, (T, C, spc, K, centre, step, L)


def _check_against_oracle(dets, x, chips, spc, freqs, tags=None, theta=None, prec="fp32"):
    L = chips.shape[1] * spc
    ref = oracle.acquire(x, chips, spc, freqs, FS, theta=theta)
    want = {r["tag"]: r for r in ref if r["detected"] and (tags is None or r["tag"] in tags)}
    got = {d.tag: d for d in dets}
    assert set(got) == set(want)
    for t, r in want.items():
        d = got[t]
        if not r["near_tie"]:
            assert (d.bin, d.lag) == (r["bin"], r["lag"])
        assert abs(d.toa - r["toa"]) <= 1e-3
        assert abs(d.peak_power - r["peak_power"]) <= 1e-9 * max(r["peak_power"], L * r["block_power"])


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("graph", [False, True])
def test_exact_bins_in_batches(dev, prec, graph):
    """Exact bins, any storage, batch (optionally graph-replayed) = single-block
    searches = the oracle at the exact frequencies."""
    chips, freqs, blocks, (T, C, spc, K, centre, step, L) = _setup(900)
    xs = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    radius = 1 if prec == "fp32" else 8
    with _plan(chips, spc, K, centre, step, 20000, 2048, exact_bins=True, precision=prec, refine_radius=radius,
               max_batch_blocks=4, graph=graph) as plan:
        assert np.array_equal(plan.freqs_hz, freqs)
        batch = plan.detect_batch(xs)
        again = plan.detect_batch(xs)
        singles = [[d for d in plan.detect(x)] for x in xs]
    key = lambda d: (d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power)   # noqa: E731
    assert [key(d) for d in batch] == [key(d) for d in again]
    for b, (x, _) in enumerate(blocks):
        mine = [d for d in batch if d.block == b]
        assert [(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in mine] == \
               [(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in singles[b]]
        _check_against_oracle(mine, x, chips, spc, freqs, prec=prec)


def test_tracking_with_exact_bins_and_16bit_storage(dev):
    """Tracking tasks on an exact-bin FP16 plan: each task equals the oracle's
    tracking task at the exact frequencies."""
    chips, freqs, blocks, (T, C, spc, K, centre, step, L) = _setup(910)
    tasks = []
    for b, (x, txs) in enumerate(blocks):
        for t in [q.tag for q in txs] + [(b * 7) % T]:
            tasks.append((x, t))
    with _plan(chips, spc, K, centre, step, 20000, 2048, exact_bins=True, precision="fp16", refine_radius=8,
               max_batch_blocks=len(tasks)) as plan:
        dets = plan.track([(torch.from_numpy(x).to(dev), t) for x, t in tasks])
    got = {d.block: d for d in dets}
    for i, (x, t) in enumerate(tasks):
        r = oracle.track(x, chips, spc, freqs, FS, t)
        if r is None or not r["detected"]:
            assert i not in got or r["near_threshold"]
            continue
        d = got[i]
        if not r["near_tie"]:
            assert (d.bin, d.lag) == (r["bin"], r["lag"])
        assert abs(d.toa - r["toa"]) <= 1e-3
        assert abs(d.peak_power - r["peak_power"]) <= 1e-9 * max(r["peak_power"], L * r["block_power"])


def test_proposal_search_on_an_exact_bin_plan(dev):
    """The proposal search on an exact-bin plan returns a subset of that plan's
    exhaustive search with identical values (the map and network do not depend
    on the bins)."""
    from paper_2005_10445_amd.proposals import LearnedParams, Network
    chips, freqs, blocks, (T, C, spc, K, centre, step, L) = _setup(920, lens=(60000, 40000))
    with _plan(chips, spc, K, centre, step, 60000, 2048, exact_bins=True) as plan, \
            Network("bf16", max_block_len=60000) as net:
        net.set_params(np.random.default_rng(3).standard_normal(net.num_params).astype(np.float32) * 0.02)
        for x, _ in blocks:
            xt = torch.from_numpy(x).to(dev)
            full = {d.tag: d for d in plan.detect(xt)}
            for kappa in (-1e9, 1e9):                 # everything proposed / nothing proposed
                dets, rep = net.detect(plan, xt, LearnedParams(kappa=kappa, max_fraction=1.0, floor_db=0.0))
                for d in dets:
                    f = full[d.tag]
                    assert (d.bin, d.lag, d.toa, d.peak_power) == (f.bin, f.lag, f.toa, f.peak_power)
                if kappa < 0:
                    assert {d.tag for d in dets} == set(full)
                else:
                    assert dets == [] and rep.segments == 0
