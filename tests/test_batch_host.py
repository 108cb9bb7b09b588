"""Host-side checks of the batch scheduler and the model autotuner (no device).

The schedule is checked against its own contract: every block goes to
exactly one team of its job's width, a team's members are distinct
workgroups on one XCD (workgroup w runs on XCD w mod 8), per-XCD residency is
respected, and the makespan stays within the longest-first bound.  The
autotuner's overlap is checked against the group-delay spread 2 pi |beta2| L
R^2 computed here independently.
"""
import math

import numpy as np
import pytest

from paper_2409_14489_amd import LinkSpec, autotune, schedule
from paper_2409_14489_amd._lib import CbessfmError


def check_schedule(jobs, spx, r):
    g = r["grid"]
    assert 0 < g <= 8 * spx
    wt, wm = r["wg_team"], r["wg_member"]
    teams = {}
    for w in range(g):
        if wt[w] < 0:
            assert wm[w] < 0
            continue
        teams.setdefault(int(wt[w]), []).append((int(wm[w]), w))
    assert len(teams) == r["n_teams"]
    width = {}
    for tm, mem in teams.items():
        members = sorted(m for m, _ in mem)
        assert members == list(range(len(mem)))               # members 0 .. w-1, each once
        assert len({w % 8 for _, w in mem}) == 1              # one XCD
        width[tm] = len(mem)
    per_xcd = np.bincount([w % 8 for w in range(g) if wt[w] >= 0], minlength=8)
    assert per_xcd.max() <= spx                                # resident
    # blocks
    it, rk = r["item_team"], r["item_rank"]
    pos = 0
    load = {tm: 0.0 for tm in teams}
    seen = {tm: [] for tm in teams}
    for w, n, c in jobs:
        for _ in range(n):
            tm = int(it[pos])
            assert width[tm] == w
            load[tm] += c
            seen[tm].append(int(rk[pos]))
            pos += 1
    for tm, ranks in seen.items():
        assert sorted(ranks) == list(range(len(ranks)))
    makespan = max(load.values())
    assert abs(makespan - r["makespan"]) <= 1e-9 * makespan
    total_area = sum(w * n * c for w, n, c in jobs)
    lb = max(max(c for _, _, c in jobs), total_area / (8 * spx))
    assert abs(r["lower_bound"] - lb) <= 1e-9 * lb
    assert r["makespan"] >= r["lower_bound"] * (1 - 1e-12)
    return makespan, lb


@pytest.mark.parametrize("seed", range(8))
def test_random_schedules_are_valid_and_balanced(seed):
    rng = np.random.default_rng(seed)
    spx = int(rng.choice([16, 32, 64]))
    jobs = []
    for _ in range(int(rng.integers(1, 60))):
        w = int(rng.integers(1, 6))
        jobs.append((w, int(rng.integers(1, 400)), float(rng.uniform(1.0, 40.0))))
    r = schedule(jobs, spx)
    makespan, lb = check_schedule(jobs, spx, r)
    # longest-first within widths: within twice the area bound plus one block
    assert makespan <= 2.0 * lb + max(c for _, _, c in jobs)


def test_uniform_jobs_fill_the_chip_evenly():
    jobs = [(5, 370, 1.0)]            # 37 blocks x 10 realisations of a 5-subband plan
    r = schedule(jobs, 32)
    check_schedule(jobs, 32, r)
    assert r["n_teams"] == 48         # 6 teams of 5 per XCD of 32 slots
    assert r["makespan"] == math.ceil(370 / 48)


def test_few_blocks_make_few_teams():
    jobs = [(3, 4, 2.0), (1, 2, 5.0)]
    r = schedule(jobs, 32)
    check_schedule(jobs, 32, r)
    assert r["n_teams"] == 6 and r["makespan"] == 5.0


def test_schedule_errors():
    with pytest.raises(CbessfmError) as e:
        schedule([(9, 3, 1.0)], 32)             # width beyond 8 subbands
    assert e.value.code == -1
    with pytest.raises(CbessfmError) as e:
        schedule([(5, 3, 1.0)], 4)              # a team does not fit one XCD
    assert e.value.code == -2
    with pytest.raises(CbessfmError) as e:
        schedule([(1, 0, 1.0)], 32)             # nothing to run
    assert e.value.code == -1
    with pytest.raises(CbessfmError) as e:
        schedule([(2, 100, 1.0)], 32, max_wg=16)
    assert e.value.code == -1


def memory_samples(beta2_ps2_km, length_km, rate):
    m = 2 * math.pi * abs(beta2_ps2_km) * 1e-24 * length_km * rate ** 2
    v = math.ceil(m)
    return v + (v & 1)


@pytest.mark.parametrize("n_sb,spans,rate", [(1, 1, 64e9), (1, 15, 64e9), (2, 5, 256e9), (5, 5, 640e9),
                                             (3, 20, 384e9)])
def test_model_autotune_covers_the_dispersion_memory(n_sb, spans, rate):
    link = LinkSpec(n_spans=spans, sample_rate_hz=rate)
    t = autotune(link, n_sb, 10, 11, 1 << 18, measure=False)
    assert t["memory"] == memory_samples(-21.7, 80.0 * spans, rate)
    assert t["measured"] == 0
    assert t["block_sb"] in [1 << k for k in range(8, 18)]
    assert t["overlap"] % 2 == 0
    assert t["covered"] == 1                        # every link here fits a block of at most 2^17
    assert t["memory"] <= t["overlap"] < n_sb * t["block_sb"]
    if t["block_sb"] > 8192:                        # streamed only when no persistent block covers
        assert t["memory"] >= n_sb * 8192
        assert t["memory"] < n_sb * t["block_sb"] and t["memory"] >= n_sb * t["block_sb"] // 2


def test_model_autotune_long_link_streams_a_covering_block():
    """40 x 80 km at 640 GS/s: memory 1.79e5 samples, beyond 5 x 8192; the
    smallest covering streamed block is N' = 2^16 (N = 327680)."""
    link = LinkSpec(n_spans=40, sample_rate_hz=640e9)
    t = autotune(link, 5, 40, 21, 1 << 20, measure=False)
    assert t["covered"] == 1 and t["block_sb"] == 1 << 16 and t["overlap"] == t["memory"]


def test_model_autotune_beyond_the_largest_block():
    """A memory beyond n_sb x 2^17 samples: the largest block, half overlap, covered = 0."""
    link = LinkSpec(n_spans=400, sample_rate_hz=640e9)
    t = autotune(link, 1, 40, 21, 1 << 22, measure=False)
    assert t["covered"] == 0 and t["block_sb"] == 1 << 17 and t["overlap"] == (1 << 17) // 2


def test_model_autotune_rejects_bad_arguments():
    link = LinkSpec()
    for args in [(0, 1, 11, 1000), (9, 1, 11, 1000), (1, 0, 11, 1000), (1, 1, 10, 1000), (1, 1, 11, 0)]:
        with pytest.raises(CbessfmError):
            autotune(link, *args, measure=False)


def test_model_autotune_memory_matches_the_overlap_the_paper_uses():
    """Sec. IV-A uses N_ov of about 1800 samples for its 15 x 80 km link
    (D = 17 ps/nm/km, i.e. beta2 = -21.68 ps^2/km at 1550 nm) sampled at
    1.125 samples per symbol of 93 GBd; the autotuner's group-delay spread of
    that link must land there."""
    d_ps_nm_km, lam, c = 17.0, 1550e-9, 299792458.0
    beta2_ps2_km = -d_ps_nm_km * 1e-6 * lam ** 2 / (2 * math.pi * c) * 1e27
    assert abs(beta2_ps2_km + 21.68) < 0.01
    link = LinkSpec(beta2_ps2_km=beta2_ps2_km, n_spans=15, sample_rate_hz=93e9 * 1.125)
    t = autotune(link, 1, 15, 11, 1 << 16, measure=False)
    assert abs(t["memory"] - 1800) <= 0.02 * 1800
