"""CPU checks of the fused kernel's launch geometry and index arithmetic.

The library's host planner (``pcal_plan`` / ``pcal_plan_launch``, no GPU
call) fixes how the fold kernel walks the stream.  These tests replay that
walk on the CPU with the kernel's own index formulas and check that

* every load stays inside the buffer and every 16-byte vector is read by
  exactly one (workgroup, thread);
* the period coordinate a thread assumes for its lanes equals the true global
  sample index modulo the fold period (the premise of the period fold);
* LDS indices, workgroup sizes and LDS bytes stay within their limits;

and that the replayed arithmetic (integer position sums, rotation by
u[q / N], fold to bins, v[b], DFT) reproduces the oracle's C_k.
"""
import numpy as np
import pytest

import oracle
import synth

pcal = pytest.importorskip("paper_2501_05993_amd.pcal")


def _levels(packed, nbits):
    b = np.asarray(packed, dtype=np.uint8)
    if nbits == 2:
        return (2 * ((b[:, None] >> np.array([0, 2, 4, 6], dtype=np.uint8)) & 3).astype(np.int64) - 3).reshape(-1)
    return b.view(np.int8).astype(np.int64)


def _walk(info, L):
    """(block, thread, vector index) of every load the fold kernel issues, in the kernel's formulas.

    Period fold: workgroup g of a tile walks groups_per_wg groups of R rows
    (one more if g < extra_groups) from group g*groups_per_wg + min(g,
    extra_groups); rows [odd_start, rows_total) go to the first workgroup of
    each tile.  Per-sample forms: rows [g*rows_per_group, +rows_per_group).
    """
    row_vecs, tile, col_tiles, W = info["row_vectors"], info["tile_vectors"], info["col_tiles"], info["period_vectors"]
    out_b, out_t, out_v = [], [], []
    rfull = L["nvec"] // row_vecs
    t = np.arange(L["threads"])
    tc, sub = t % tile, t // tile

    def emit(blk, r, tmask):
        c = blk % col_tiles
        colp = c * tile + tc
        colr = colp + sub * W
        ok = tmask & (colp < W) & (colr < row_vecs) & ((r < rfull) | ((r == rfull) & (colr < L["nvec"] - rfull * row_vecs)))
        tt = t[ok]
        out_b.append(np.full(tt.size, blk))
        out_t.append(tt)
        out_v.append(r * row_vecs + colr[ok])

    every = np.ones(t.size, bool)
    fold = info["method"] == pcal.METHOD_PERIOD_FOLD
    for blk in range(L["grid"]):
        g = blk // col_tiles
        if fold:
            R = L["R"]
            r0 = R * (g * L["groups_per_wg"] + min(g, L["extra_groups"]))
            r1 = r0 + R * (L["groups_per_wg"] + (1 if g < L["extra_groups"] else 0))
            assert r1 <= rfull
        else:
            r0 = g * L["rows_per_group"]
            r1 = min(r0 + L["rows_per_group"], L["rows_total"])
        for r in range(r0, r1):
            emit(blk, r, every)
    if fold:
        for c in range(col_tiles):  # rows after the last whole group: first workgroup of the tile
            for r in range(L["odd_start"], L["rows_total"]):
                emit(c, r, every)
    if not out_v:
        return np.zeros(0, int), np.zeros(0, int), np.zeros(0, int)
    return np.concatenate(out_b), np.concatenate(out_t), np.concatenate(out_v)


def _geometry(fs, fc, fo, nbits, nsamples, addr_low=0, before=0, method=0):
    info = pcal.plan(fs, fc, fo, nbits, method=method)
    L = pcal.plan_launch(fs, fc, fo, nbits, nsamples, addr_low=addr_low, samples_before=before, method=method)
    spv = (64 if nbits == 2 else 16) if info["method"] == pcal.METHOD_PERIOD_FOLD else 16
    L["tile_vecs"] = info["tile_vectors"]
    L["pos_cols"] = info["tile_vectors"]
    L["R"] = 5 if nbits == 2 else 4  # rows per walker group of the period fold
    return info, L, spv


CASES = [
    # fs, f_comb, f_offset, nbits, nsamples, addr_low, samples_before
    (32_000_000, 1_000_000, 0, 2, 4 * 100_003, 0, 0),
    (64_000_000, 1_000_000, 10_000, 2, 4 * 400_011, 0, 0),
    (64_000_000, 1_000_000, 10_000, 2, 4 * 300_000, 5, 4 * 777),
    (1_024_000_000, 1_000_000, 510_000, 8, 1_000_003, 0, 0),
    (1_024_000_000, 1_000_000, 510_000, 8, 2_000_000, 9, 123_457),
    (512_000_000, 1_000_000, 10_000, 2, 4 * 250_001, 3, 4 * 51),
    (16_000_000, 1_000_000, 250_000, 2, 4 * 50_000, 0, 0),
    (24_000_000, 1_000_000, 500_000, 8, 333_333, 1, 17),
    (64_000_000, 1_000_000, 10_000, 2, 4 * 9, 3, 0),        # head and tail only
    (32_000_000, 1_000_000, 0, 8, 7, 2, 5),                  # fewer samples than one vector
]


@pytest.mark.parametrize("fs,fc,fo,nbits,ns,addr,before", CASES)
def test_walk_bounds_coverage_and_period(fs, fc, fo, nbits, ns, addr, before):
    info, L, spv = _geometry(fs, fc, fo, nbits, ns, addr, before)
    spb = 8 // nbits
    Sp = info["fold_period"]
    assert L["head_bytes"] + 16 * L["nvec"] + L["tail_bytes"] == ns // spb
    assert L["head_bytes"] == min((16 - addr % 16) % 16, ns // spb)
    assert 0 <= L["tail_bytes"] < 16
    assert L["threads"] % 64 == 0 and L["threads"] <= 1024
    assert L["threads"] >= L["tile_vecs"]
    assert L["lds_bytes"] <= 65536
    assert info["lds_positions"] <= 12800
    npos_sk = info["lds_positions"] + info["lds_positions"] // spv     # skewed position sums
    assert L["lds_bytes"] >= 4 * npos_sk and L["lds_bytes"] >= 40 * L["threads"]
    assert info["row_vectors"] * spv % Sp == 0          # rows are whole fold periods
    blk, thr, vec = _walk(info, L)
    # in bounds, each vector exactly once
    assert vec.size == L["nvec"]
    if vec.size:
        assert vec.min() >= 0 and vec.max() < L["nvec"]
        assert np.unique(vec).size == vec.size
    # the period coordinate each thread assumes equals the true one
    g0 = before + L["head_bytes"] * spb
    c = blk % info["col_tiles"]
    qb = (L["q0"] + c * L["tile_vecs"] * spv) % Sp
    assumed = (qb + (thr % L["pos_cols"]) * spv) % Sp
    true = (g0 + vec * spv) % Sp
    np.testing.assert_array_equal(assumed, true)
    assert np.all((thr % L["pos_cols"]) * spv + spv <= info["lds_positions"])
    assert np.all((thr % L["pos_cols"]) * (spv + 1) + spv - 1 < npos_sk)  # skewed LDS index in range
    assert L["q0"] == g0 % Sp and L["head_q"] == before % Sp
    assert L["tail_q"] == (g0 + L["nvec"] * spv) % Sp


@pytest.mark.parametrize("fs,fc,fo,nbits,ns", [
    (64_000_000, 1_000_000, 10_000, 2, 1 << 30),
    (32_000_000, 1_000_000, 0, 2, 1 << 24),
    (1_024_000_000, 1_000_000, 510_000, 8, 1 << 28),
    (512_000_000, 1_000_000, 510_000, 2, 1 << 26),
    (16_000_000, 1_000_000, 10_000, 2, 1 << 26),
])
def test_full_size_launch_limits(fs, fc, fo, nbits, ns):
    info, L, spv = _geometry(fs, fc, fo, nbits, ns)
    ngroups = L["grid"] // info["col_tiles"]
    unit = 5 if nbits == 2 else 4
    rfull = L["nvec"] // info["row_vectors"]
    wgroups = rfull // unit
    assert L["grid"] >= 1 and ngroups * L["groups_per_wg"] + L["extra_groups"] == wgroups
    assert 0 <= L["extra_groups"] < ngroups and L["odd_start"] == wgroups * unit
    assert L["rows_total"] - L["odd_start"] <= unit  # at most unit - 1 full rows and a partial one
    assert ngroups == 1 or L["groups_per_wg"] >= 1
    assert L["threads"] <= 1024 and L["lds_bytes"] <= 65536
    assert L["nvec"] * 16 + L["head_bytes"] + L["tail_bytes"] == ns * nbits // 8


def _emulate(packed, nbits, ns, fs, fc, fo, addr, before):
    """The fold kernel's arithmetic replayed in numpy FP64 (position sums -> u -> bins -> v -> DFT)."""
    info, L, spv = _geometry(fs, fc, fo, nbits, ns, addr, before)
    spb = 8 // nbits
    N, Sp = fs // fc, info["fold_period"]
    M = Sp // N
    x = _levels(packed, nbits)[:ns]
    nh = L["head_bytes"] * spb
    u = np.exp(-2j * np.pi * ((fo * N * np.arange(M)) % fs) / fs)
    v = np.exp(-2j * np.pi * ((fo * np.arange(N)) % fs) / fs)
    blk, thr, vec = _walk(info, L)
    Q = np.zeros(N, complex)
    for b in np.unique(blk):
        sel = blk == b
        F = np.zeros(info["lds_positions"], np.int64)
        for s in range(spv):
            np.add.at(F, (thr[sel] % L["pos_cols"]) * spv + s, x[nh + vec[sel] * spv + s])
        c = b % info["col_tiles"]
        qb = (L["q0"] + c * L["tile_vecs"] * spv) % Sp
        q = (qb + np.arange(F.size)) % Sp
        np.add.at(Q, q % N, F * u[q // N])
    for start, n, q0 in ((0, nh, L["head_q"]), (nh + L["nvec"] * spv, L["tail_bytes"] * spb, L["tail_q"])):
        q = (q0 + np.arange(n)) % Sp
        np.add.at(Q, q % N, x[start:start + n] * u[q // N])
    P = v * Q
    k = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(k, k) / N) @ P


@pytest.mark.parametrize("fs,fc,fo,nbits,ns,addr,before", [c for c in CASES if c[4] <= 4 * 400_011])
def test_emulated_arithmetic_matches_oracle(fs, fc, fo, nbits, ns, addr, before):
    spec = synth.CombSpec(fs, fc, fo, nbits, amp=0.3 if nbits == 2 else 4.0, t_d=5e-9,
                          sigma=1.0 if nbits == 2 else 20.0, seed=(77, ns))
    packed = synth.make_stream(spec, ns + (-ns) % (8 // nbits))
    got = _emulate(packed, nbits, ns, fs, fc, fo, addr, before)
    want = oracle.correlate(packed, nbits, ns, fs, fc, fo, n0=before)
    scale = max(1.0, np.abs(want).max())
    assert np.max(np.abs(got - want)) <= 1e-9 * scale


# ---------------------------------------------------------------- per-sample forms (table / recurrence)

ROT_CASES = [
    (1_024_000_000, 1_000_000, 510_000, 8, 1_000_003, 0, 0),
    (1_024_000_000, 1_000_000, 510_000, 8, 3_000_000, 9, 123_457),
    (64_000_000, 1_000_000, 10_000, 2, 4 * 300_001, 1, 4 * 77),
    (64_000_000, 2_000_000, 10_007, 8, 555_555, 5, 10 ** 9 + 7),    # prime offset
    (24_000_000, 1_000_000, 500_000, 2, 4 * 5, 3, 0),               # head and tail only
    (48_000_000, 1_000_000, 250_000, 8, 200_000, 0, 3),             # N = 48: rows of lcm(48, 16)
]


@pytest.mark.parametrize("method", [2, 3, 5])
@pytest.mark.parametrize("fs,fc,fo,nbits,ns,addr,before", ROT_CASES)
def test_per_sample_walk(method, fs, fc, fo, nbits, ns, addr, before):
    if method == 2 and fo == 10_007:
        with pytest.raises(pcal.PcalError):   # rotator period fs: no table
            pcal.plan(fs, fc, fo, nbits, method=method)
        return
    info, L, spv = _geometry(fs, fc, fo, nbits, ns, addr, before, method=method)
    assert info["method"] == method
    N = fs // fc
    spb = 8 // nbits
    vb = 16 // spb                                   # bytes per thread-vector of 16 samples
    assert L["head_bytes"] == min((vb - addr % vb) % vb, ns // spb)
    assert L["head_bytes"] + vb * L["nvec"] + L["tail_bytes"] == ns // spb
    assert 0 <= L["tail_bytes"] < vb
    assert L["threads"] <= 512 and L["threads"] % 64 == 0 and L["threads"] >= L["tile_vecs"]
    assert L["lds_bytes"] == 16 * N
    assert (info["row_vectors"] * 16) % N == 0       # every lane keeps its bin
    assert info["row_vectors"] % info["period_vectors"] == 0
    blk, thr, vec = _walk(info, L)
    assert vec.size == L["nvec"]
    if vec.size:
        assert vec.min() >= 0 and vec.max() < L["nvec"] and np.unique(vec).size == vec.size
        g0 = before + L["head_bytes"] * spb
        c = blk % info["col_tiles"]
        colr = c * L["tile_vecs"] + thr % L["tile_vecs"] + (thr // L["tile_vecs"]) * info["period_vectors"]
        # bin the kernel assigns to lane 0 == true bin of the sample
        np.testing.assert_array_equal((g0 + colr * 16) % N, (g0 + vec * 16) % N)
    assert L["q0"] == before + L["head_bytes"] * spb
    assert L["head_q"] == before and L["tail_q"] == L["q0"] + 16 * L["nvec"]


def test_auto_prefers_recurrence_for_long_periods():
    """AUTO folds up to a 2^23-sample fold period and takes the recurrence beyond."""
    assert pcal.plan(64_000_000, 1_000_000, 10_000, 2)["method"] == pcal.METHOD_PERIOD_FOLD
    p = pcal.plan(64_000_000, 1_000_000, 10_008, 2)  # R = 8e6 <= 2^23
    assert p["fold_period"] == 8_000_000 and p["method"] == pcal.METHOD_PERIOD_FOLD
    p = pcal.plan(64_000_000, 1_000_000, 10_004, 2)  # R = 16e6 > 2^23
    assert p["fold_period"] == 16_000_000 and p["method"] == pcal.METHOD_OSC
    assert pcal.plan(64_000_000, 2_000_000, 10_007, 8)["method"] == pcal.METHOD_OSC


# fs, f_offset, nbits across the paper's and the serving mix's configurations
_PLAN_CASES = [(fs * 1_000_000, fo, nb) for fs in (16, 32, 64, 128, 256, 512, 1024)
               for fo in (0, 10_000, 250_000, 500_000, 510_000) for nb in (2, 8)]
# long fold periods: 625 and 5000 column tiles at 2-bit
_PLAN_CASES += [(64_000_000, 10_008, 2), (64_000_000, 10_007, 2), (64_000_000, 10_008, 8)]


@pytest.mark.parametrize("fs,fo,nbits", _PLAN_CASES)
def test_fold_plan_rules(fs, fo, nbits):
    """The planner's fold geometry: the fold period is a multiple of the joint
    period and of one vector, at least 64 vectors long (a wave's lanes own
    distinct positions) and the first such multiple; split tiles are whole
    128-byte lines wide and hold at most 12800 positions; workgroups are at
    least 448 threads, waste the fewest lanes, and among equal sizes take the
    one nearest 640 -- except for a period split into more than 256 tiles,
    whose workgroups are the smallest multiple of 64 threads that covers one
    tile (one row of the tile each)."""
    info = pcal.plan(fs, 1_000_000, fo, nbits, method=pcal.METHOD_PERIOD_FOLD)
    spv = 64 if nbits == 2 else 16
    S, Sp = info["joint_period"], info["fold_period"]
    base = int(np.lcm(S, spv))
    assert Sp % base == 0 and Sp % spv == 0
    W = Sp // spv
    assert W >= 64 and (Sp == base or (Sp - base) // spv < 64)
    assert info["period_vectors"] == W
    tile, tiles, thr = info["tile_vectors"], info["col_tiles"], info["block_threads"]
    assert tile * tiles >= W and tile * (tiles - 1) < W
    assert info["lds_positions"] == tile * spv <= 12800
    if tiles > 1:
        assert tile % 8 == 0
    if tiles > 256:
        assert thr == (tile + 63) // 64 * 64 and info["row_vectors"] == W
        return
    assert 448 <= thr <= 768 and thr % 64 == 0 and thr >= tile
    eff = lambda t: (t // tile) * tile / t
    best = max(eff(t) for t in range(448, 769, 64) if t >= tile)
    assert abs(eff(thr) - best) < 1e-9
    ties = [t for t in range(448, 769, 64) if t >= tile and abs(eff(t) - best) < 1e-9]
    assert abs(thr - 640) == min(abs(t - 640) for t in ties)
    assert info["row_vectors"] == (thr // tile) * W if tiles == 1 else info["row_vectors"] % W == 0


@pytest.mark.parametrize("fs,fc,fo", [(1_024_000_000, 1_000_000, 250_010), (64_000_000, 1_000_000, 15_626),
                                      (64_000_000, 2_000_000, 10_007), (1_024_000_000, 1_000_000, 510_000),
                                      (512_000_000, 1_000_000, 125_003), (48_000_000, 1_000_000, 250_001)])
@pytest.mark.parametrize("prec", [pcal.PREC_F64, pcal.PREC_MIXED])
def test_resonator_row_step_far_from_zero_and_pi(fs, fc, fo, prec):
    """The resonator steps by d = w_o * (samples per row) with 2 cos d rounded: the planner picks the
    row length (sub-rows of lcm(N, 16) samples, 256-512-thread workgroups) whose |sin d| is largest up
    to 0.2, the smallest workgroup among those, wasting no more lanes than the others."""
    info = pcal.plan(fs, fc, fo, 8, method=pcal.METHOD_OSC, precision=prec)
    N = fs // fc
    per = int(np.lcm(N, 16))
    W = per // 16
    dn = info["row_vectors"] * 16
    assert dn % per == 0

    def score(t):
        k = t // W
        return min(abs(np.sin(2 * np.pi * ((fo * k * per) % fs) / fs)), 0.2)
    cands = [t for t in range(256, 513, 64) if t >= W]
    best = max(score(t) for t in cands)
    assert abs(score(info["block_threads"]) - best) < 1e-12
    assert min(abs(np.sin(2 * np.pi * ((fo * dn) % fs) / fs)), 0.2) == pytest.approx(best, abs=1e-12)
    assert best >= 0.2


def test_auto_takes_coupled_form_when_no_row_step_suits_the_resonator():
    """f_offset = 1000001 Hz at fs = 1024 MHz: the rotator advances by 2 pi 1e-6 per 1024 samples, so every
    row length leaves d near 0.  AUTO keeps the resonator in FP64 (its coefficient error is 2^-29 of
    FP32's) and takes the coupled form in the FP32-state forms."""
    assert pcal.plan(1_024_000_000, 1_000_000, 1_000_001, 8, precision=pcal.PREC_F64)["method"] == pcal.METHOD_OSC
    for prec in (pcal.PREC_MIXED, pcal.PREC_F32):
        assert pcal.plan(1_024_000_000, 1_000_000, 1_000_001, 8, precision=prec)["method"] == pcal.METHOD_CFO
    # an offset whose row step suits the resonator keeps it in every form
    for prec in (pcal.PREC_F64, pcal.PREC_MIXED, pcal.PREC_F32):
        assert pcal.plan(64_000_000, 2_000_000, 10_007, 8, precision=prec)["method"] == pcal.METHOD_OSC
