"""Parity of the HIP sort (called through the C ABI) with the CPU oracle.

Keys must be bit-identical to the oracle's sorted keys; records must also
keep their multiset.  Sizes span several blocks, stripes and a ragged tail.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_2009_13569_amd as ips
import synth
from gpu_util import assert_parity, generate, gpu_sort, log

pytestmark = pytest.mark.gpu

KINDS = ["u32", "u64", "f64", "pair", "rec100", "quartet"]


def _quartet_of(v: np.ndarray) -> np.ndarray:
    """Quartets whose (a, b, c) keys are ordered as v: a fixed, v split over
    the top bits of b and c (so that neighbouring keys differ in c and keys
    far apart in b), the value the position."""
    n = v.size
    v = v.astype(np.uint64)
    out = np.empty((n, 4), dtype=np.uint64)
    out[:, 0] = np.uint64(0x5A01_0203_0405_0607)
    out[:, 1] = v >> np.uint64(6)
    out[:, 2] = ((v & np.uint64(63)) << np.uint64(58)) | np.uint64(0x1234)
    out[:, 3] = np.arange(n, dtype=np.uint64)
    return out


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0)


@pytest.fixture(scope="module")
def untuned():
    """A sorter without the tuning table: the root step runs exactly the
    parameters the test gives (k = 256 unless set), as the oracle assumes."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0, tuning=None)


@pytest.mark.parametrize("kind", KINDS)
def test_lds_tier(sorter, kind):
    cap = ips.LDS_CAP[kind]
    for n in sorted({2, 3, 17, 33, 1000, cap // 4, cap // 4 + 1, cap // 2, cap // 2 + 1, cap - 1, cap}):
        a = generate(kind, "uniform", n, 100 + n)
        log(f"lds {kind} n={n}")
        assert_parity(gpu_sort(sorter, a, kind), a, kind)


def _narrow_dup_input(kind: str, n: int, pairs: int, gap: int, seed: int) -> np.ndarray:
    """n elements whose keys take 2 * pairs values: for i < pairs, base +
    128 i and base + 128 i + gap, each element picking one at random.  Over
    a span of 128 * pairs values the binning of a single LDS-tier task puts
    both values of a pair into one bin of a few dozen to about 130 keys (a
    bin spanning at most 64 possible values)."""
    x = synth.stream(seed, n)
    i = (x % np.uint64(pairs)).astype(np.uint64)
    v = i * np.uint64(128) + ((x >> np.uint64(32)) & np.uint64(1)) * np.uint64(gap)
    if kind == "u32":
        return (v + np.uint64(0x9000_0000)).astype(np.uint32)
    if kind == "u64":
        return v + np.uint64(0x1234_5678_9000_0000)
    if kind == "f64":   # positive doubles: the bit pattern orders them
        return (v + np.uint64(0x4100_0000_0000_0000)).view(np.float64)
    if kind == "pair":
        out = np.empty((n, 2), dtype=np.uint64)
        out[:, 0] = v + np.uint64(0x1234_5678_9000_0000)
        out[:, 1] = np.arange(n, dtype=np.uint64)
        return out
    if kind == "quartet":
        return _quartet_of(v)
    out = synth.gen_rec100("uniform", n, seed)     # payload and index from the generator
    out[:, 0:8] = np.frombuffer(bytes([0x5A, 1, 2, 3, 4, 5, 6, 7]), dtype=np.uint8)
    out[:, 8:10] = v.astype(">u2").view(np.uint8).reshape(n, 2)
    return out


@pytest.mark.parametrize("kind", KINDS)
def test_lds_tier_narrow_duplicate_bins(sorter, kind):
    """Bins of 17 to about 130 keys holding two values within a window of
    at most 64 values (what duplicate-heavy inputs such as TwoDup give the
    LDS tier): they are sorted by the wavefront counting sort, those above
    the wavefront limit by another binning round."""
    n = {"pair": 4000, "rec100": 1000}.get(kind, 4000)
    gap = 5 if kind == "rec100" else 3
    for pairs in (16, 32, 64):
        a = _narrow_dup_input(kind, n, pairs, gap, 4242 + pairs)
        log(f"lds narrow dup {kind} pairs={pairs}")
        assert_parity(gpu_sort(sorter, a, kind, params=ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)), a, kind)


def _keyed(kind: str, v: np.ndarray, seed: int) -> np.ndarray:
    """Elements of `kind` whose keys are base + v, in key order of v (v <
    2^16 for records, whose key ends in v as two bytes); records get their
    payload from the generator."""
    n = v.size
    v = v.astype(np.uint64)
    if kind == "u32":
        return (v + np.uint64(0x9000_0000)).astype(np.uint32)
    if kind == "u64":
        return v + np.uint64(0x1234_5678_9000_0000)
    if kind == "f64":   # positive doubles: the bit pattern orders them
        return (v + np.uint64(0x4100_0000_0000_0000)).view(np.float64)
    if kind == "pair":
        out = np.empty((n, 2), dtype=np.uint64)
        out[:, 0] = v + np.uint64(0x1234_5678_9000_0000)
        out[:, 1] = np.arange(n, dtype=np.uint64)
        return out
    if kind == "quartet":
        return _quartet_of(v)
    out = synth.gen_rec100("uniform", n, seed)
    out[:, 0:8] = np.frombuffer(bytes([0x5A, 1, 2, 3, 4, 5, 6, 7]), dtype=np.uint8)
    out[:, 8:10] = v.astype(">u2").view(np.uint8).reshape(n, 2)
    return out


@pytest.mark.parametrize("kind", KINDS)
def test_lds_tier_clustered_bins(sorter, kind):
    """Keys in narrow clusters spread over a wide range: the binning of one
    LDS-tier task gives bins of 17 to about 100 keys holding many values
    (wider than the counting sort's 64), sorted by the wavefront register
    network with one or two keys per lane."""
    n, clusters, width, spacing = {"rec100": (1000, 12, 300, 3000)}.get(kind, (4000, 48, 150, 1400))
    for seed in (11, 12):
        x = synth.stream(seed, 2 * n)
        v = (x[0::2] % np.uint64(clusters)) * np.uint64(spacing) + (x[1::2] % np.uint64(width))
        a = _keyed(kind, v, seed)
        log(f"lds clustered {kind} seed={seed}")
        assert_parity(gpu_sort(sorter, a, kind, params=ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)), a, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_lds_tier_sorted_reverse_repeated(sorter, kind):
    """Sorted and reverse inputs whose last keys sit in a partly filled
    register slot, each sorted many times.  A 64-bit shift reading its amount
    from outside the wavefront's register allocation once gave one
    wavefront's keys wrong bins in about one run in ten for such inputs (u64,
    5000 and 5832 keys); the kernels now build those shifts from 32-bit
    operations."""
    cap = {"u32": 16384, "u64": 16384, "f64": 16384, "pair": 8192}[kind]
    flags = ips.FLAG_NO_SORTED_CHECK
    for n in (5000, 5832, int(cap * 0.3) + 7, int(cap * 0.7) + 3):
        n = min(n, cap)
        base = generate(kind, "uniform", n, 7 + n)
        ref = oracle.sort(base, kind)
        for name, a in (("sorted", ref), ("reverse", ref[::-1].copy())):
            log(f"lds repeat {kind} {name} n={n}")
            for _ in range(12):
                assert_parity(gpu_sort(sorter, a, kind, params=ips.make_params(flags=flags)), a, kind, ref)


DISTS = {
    "u32": ["uniform", "exponential", "rootdup", "twodup", "eightdup", "almostsorted", "zipf"],
    "u64": ["uniform", "exponential", "rootdup", "twodup", "eightdup", "almostsorted", "zipf"],
    "f64": ["uniform", "exponential"],
    "pair": ["uniform", "rootdup"],
    "rec100": ["uniform", "rootdup"],
    "quartet": ["uniform", "rootdup", "eightdup"],
}


@pytest.mark.parametrize("kind", KINDS)
def test_samplesort_parity(sorter, kind):
    nbig = {"rec100": 40_000, "quartet": 150_001}.get(kind, 300_001)
    for dist in DISTS[kind]:
        for n in (20_011, nbig):
            a = generate(kind, dist, n, 7)
            log(f"samplesort {kind} {dist} n={n}")
            p = ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)
            assert_parity(gpu_sort(sorter, a, kind, params=p), a, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_radix_parity(sorter, kind):
    for dist in DISTS[kind]:
        for n in (20_011, 300_001):
            a = generate(kind, dist, n, 9)
            log(f"radix {kind} {dist} n={n}")
            assert_parity(gpu_sort(sorter, a, kind, algo="radix"), a, kind)


def test_config1_full(sorter):
    """n = 2^20 uniform u64, k = 256, 2 KiB blocks, n0 = 16."""
    a = synth.gen_u64("uniform", 1 << 20, synth.seed_for(1))
    p = ips.make_params(k=256, block_bytes=2048, n0=16, flags=ips.FLAG_GLOBAL_BUFFERS)
    log("config1 gbuf")
    assert_parity(gpu_sort(sorter, a, "u64", params=p), a, "u64")
    log("config1 lds")
    assert_parity(gpu_sort(sorter, a, "u64"), a, "u64")


def _level1(sorter, a, kind, params, algo="samplesort"):
    out = gpu_sort(sorter, a, kind, algo=algo, params=params)
    ri = sorter.root_info()
    assert ri.valid == 1
    return out, ri


LDS_CAP = ips.LDS_CAP


@pytest.mark.parametrize("kind,n,gbuf,n0", [("u64", 1 << 20, True, 16), ("u64", 1 << 20, False, 16),
                                            ("u32", 300_001, False, 16), ("f64", 200_003, False, 16),
                                            ("pair", 100_003, False, 16), ("rec100", 30_011, False, 16),
                                            ("u64", 300_001, False, 0), ("rec100", 30_011, False, 0),
                                            ("quartet", 100_003, False, 16), ("quartet", 60_011, False, 0)])
def test_level1_exact(untuned, kind, n, gbuf, n0):
    """The root step's sample, splitters, equality-bucket flag and bucket
    boundaries equal the oracle's, and every element lies in its bucket.
    n0 = 0 checks the default base-case size (a quarter of the LDS tier)."""
    for dist in ("uniform", "rootdup"):
        a = generate(kind, dist, n, 3)
        flags = ips.FLAG_LEVEL1_ONLY | ips.FLAG_PAPER_ROOT_ALPHA | (ips.FLAG_GLOBAL_BUFFERS if gbuf else 0)
        p = ips.make_params(block_bytes=2048 if gbuf else 0, flags=flags, seed=12345, n0=n0)
        log(f"level1 {kind} {dist} n={n} gbuf={gbuf} n0={n0}")
        out, ri = _level1(untuned, a, kind, p)
        if n0:
            st = oracle.sample_step(a, kind, seed=12345, n0=n0)
        else:
            # default k': smallest power of two (<= 256) with mean bucket <= cap/4
            kp = 2
            while kp < 256 and kp * (LDS_CAP[kind] // 4) < n:
                kp *= 2
            assert ri.k_prime == kp
            st = oracle.sample_step(a, kind, seed=12345, k=kp, n0=1)
        assert (ri.alpha, ri.k_prime, ri.m, ri.u, ri.K, bool(ri.eq), ri.nb) == \
            (st["alpha"], st["k_prime"], st["m"], st["u"], st["K"], st["eq"], st["nb"])
        spl = st["splitters"]
        for i in range(st["K"]):
            got = bytes(ri.splitters[i])
            if kind == "rec100":
                assert got[:10] == bytes(spl[i][:10]), i
            elif kind == "quartet":      # words a and b are reported
                assert got == np.ascontiguousarray(spl[i][:2]).tobytes(), i
            elif kind == "u32":
                assert int.from_bytes(got[:8], "little") == int(spl[i]), i
            else:
                assert got[:8] == np.ascontiguousarray(spl[i]).tobytes()[:8], i
        hist = oracle.histogram(a, kind, spl, st["K"], st["eq"])
        starts = np.concatenate([[0], np.cumsum(hist)]).astype(np.uint64)
        assert np.array_equal(np.array(ri.bucket_start[:st["nb"] + 1], dtype=np.uint64), starts)
        assert oracle.check_partition(out, kind, spl, st["K"], st["eq"], starts) is None
        assert_parity(oracle.sort(out, kind), a, kind)     # multiset kept


@pytest.mark.parametrize("kind", ["u32", "u64", "pair"])
def test_level1_radix_exact(untuned, kind):
    for dist in ("uniform", "rootdup", "exponential"):
        a = generate(kind, dist, 200_003, 5)
        log(f"level1 radix {kind} {dist}")
        out, ri = _level1(untuned, a, kind, ips.make_params(flags=ips.FLAG_LEVEL1_ONLY), "radix")
        d = oracle.radix_digit_info(a, kind)
        assert (ri.radix_shift, ri.radix_width) == (d["shift"], d["width"])
        h = oracle.radix_histogram(a, kind, d["shift"], d["width"])
        starts = np.concatenate([[0], np.cumsum(h)]).astype(np.uint64)
        assert np.array_equal(np.array(ri.bucket_start[:ri.nb + 1], dtype=np.uint64), starts)
        keys = out if kind != "pair" else out[:, 0]
        dig = (keys.astype(np.uint64) >> np.uint64(d["shift"])) & np.uint64((1 << d["width"]) - 1)
        assert np.all(np.diff(dig.astype(np.int64)) >= 0)


@pytest.mark.parametrize("k,bb", [(2, 8), (4, 8), (2, 16), (4, 16)])
def test_brute_force_tiny(sorter, k, bb):
    """Every permutation of distinct keys and every sequence over {0,1,2}
    (n <= 6), through the partitioning path (LDS tier off)."""
    base = dict(k=k, block_bytes=bb, n0=1, lds_task_max=1, flags=ips.FLAG_NO_SORTED_CHECK)
    for eqflag in (0, ips.FLAG_EQ_ON, ips.FLAG_EQ_OFF):
        p = ips.make_params(**{**base, "flags": base["flags"] | eqflag})
        for n in range(2, 7):
            log(f"brute k={k} bb={bb} eq={eqflag} n={n}")
            vals = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15 >> 3)
            for perm in itertools.permutations(range(n)):
                a = vals[list(perm)]
                assert np.array_equal(gpu_sort(sorter, a, "u64", params=p), np.sort(vals)), perm
            if n <= 5:
                for seq in itertools.product(range(3), repeat=n):
                    a = np.array(seq, dtype=np.uint64)
                    assert np.array_equal(gpu_sort(sorter, a, "u64", params=p), np.sort(a)), seq


@pytest.mark.parametrize("kind", KINDS)
def test_edge_cases(sorter, kind):
    rng = np.random.default_rng(11)
    p1 = ips.make_params(lds_task_max=1, flags=ips.FLAG_NO_SORTED_CHECK)
    for n in (0, 1, 2, 63, 64, 65, 127, 128, 129, 193, 1000, 4097):
        a = generate(kind, "uniform", n, 200 + n)
        log(f"edge {kind} n={n}")
        assert_parity(gpu_sort(sorter, a, kind, params=p1), a, kind)
        assert_parity(gpu_sort(sorter, a, kind), a, kind)
    n = 70_001
    base = generate(kind, "uniform", n, 1)
    cases = {"all_equal": np.repeat(base[:1], n, axis=0),
             "two_values": base[rng.integers(0, 2, n)],
             "one_outlier": np.concatenate([np.repeat(base[:1], n - 1, axis=0), base[1:2]])}
    s = oracle.sort(base, kind)
    cases["sorted"] = s
    cases["reverse"] = s[::-1].copy()
    for name, a in cases.items():
        for params in (None, ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)):
            log(f"edge {kind} {name} check={params is None}")
            assert_parity(gpu_sort(sorter, np.ascontiguousarray(a), kind, params=params), a, kind)


def test_extreme_keys(sorter):
    n = 50_000
    rng = np.random.default_rng(3)
    u = rng.choice(np.array([0, 1, 2**63, 2**64 - 2, 2**64 - 1], dtype=np.uint64), n)
    for algo in ("samplesort", "radix"):
        log(f"extreme u64 {algo}")
        assert_parity(gpu_sort(sorter, u, "u64", algo=algo), u, "u64")
    specials = np.array([0x0, 0x8000000000000000, 0x1, 0x8000000000000001, 0x7FF0000000000000,
                         0xFFF0000000000000, 0x3FF0000000000000, 0xBFF0000000000000,
                         0x7FF8000000000000, 0xFFF8000000000000], dtype=np.uint64)
    f = specials[rng.integers(0, specials.size, n)].view(np.float64)
    for algo in ("samplesort", "radix"):
        log(f"extreme f64 {algo}")
        out = gpu_sort(sorter, f, "f64", algo=algo)
        assert np.array_equal(out.view(np.uint64), oracle.sort(f, "f64").view(np.uint64))
    r = synth.gen_rec100("uniform", 20_000, 4)
    r[::3, 0] = 0xFF
    r[1::3, 0] = 0x80
    log("extreme rec100")
    assert_parity(gpu_sort(sorter, r, "rec100"), r, "rec100")


def _pattern_u64(name, n, rng):
    u = rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    if name == "clustered":          # one bin far above the wavefront limit
        m = int(n * 0.8)
        u[:m] = rng.integers(0, 100, m, dtype=np.uint64)
    elif name == "mid_cluster":      # one bin of a few hundred keys
        u[:300] = np.uint64(1 << 62) + rng.integers(0, 1000, 300, dtype=np.uint64)
    elif name == "three_values":
        u = rng.integers(0, 3, n, dtype=np.uint64) * np.uint64(1 << 40)
    elif name == "all_equal":
        u[:] = np.uint64(12345)
    rng.shuffle(u)
    return u


def _as_kind(u, kind):
    n = u.size
    if kind == "u64":
        return u
    if kind == "u32":
        return (u >> np.uint64(32)).astype(np.uint32)
    if kind == "f64":
        return (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    if kind == "pair":
        return np.stack([u, np.arange(n, dtype=np.uint64)], axis=1)
    if kind == "quartet":       # u in word b, a shared, c a function of u
        return np.stack([np.full(n, 7, dtype=np.uint64), u, ~u, np.arange(n, dtype=np.uint64)], axis=1)
    r = synth.gen_rec100("uniform", n, 5)
    r[:, 0:2] = 0
    r[:, 2:10] = u.astype(">u8").view(np.uint8).reshape(n, 8)
    return r


@pytest.mark.parametrize("kind", KINDS)
def test_lds_tier_fallbacks(sorter, kind):
    """Bins above the register-network size, above the wavefront limit, few
    distinct keys and all-equal keys inside single LDS-tier tasks."""
    rng = np.random.default_rng(21)
    cap = ips.LDS_CAP[kind]
    for name in ("clustered", "mid_cluster", "three_values", "all_equal"):
        for n in sorted({cap // 2 + 7, cap}):
            a = _as_kind(_pattern_u64(name, n, rng), kind)
            log(f"lds fallback {kind} {name} n={n}")
            p = ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)
            assert_parity(gpu_sort(sorter, a, kind, params=p), a, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_presorted_inputs_through_partitioning(sorter, kind):
    # Sorted and reverse-sorted inputs with the detection switched off go
    # through the partitioning steps (as segments of a batched call do).
    p = ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK)
    for dist in ("sorted", "reversesorted", "zero"):
        for n in (20_011, 300_001):
            a = generate(kind, dist, n, 11)
            for algo in ("samplesort", "radix"):
                log(f"presorted {kind} {dist} n={n} {algo}")
                assert_parity(gpu_sort(sorter, a, kind, algo=algo, params=p), a, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "pair", "rec100", "quartet"])
def test_block_sizes(kind):
    """Every block size the parameters allow (which sets how many lanes move
    one block in the permutation: 4 to 64) sorts like the oracle, on inputs
    that need two partitioning levels.  2 KiB blocks need global buffers."""
    s = ips.Sorter(0, tuning=None)
    n = {"u32": 3_000_017, "u64": 2_100_001, "pair": 600_011, "rec100": 120_007, "quartet": 300_007}[kind]
    a = generate(kind, "uniform", n, 4242)
    ref = oracle.sort(a, kind)
    for bb in (128, 256, 512, 1024, 2048):
        flags = ips.FLAG_GLOBAL_BUFFERS if bb == 2048 else 0
        p = ips.make_params(block_bytes=bb, flags=flags | ips.FLAG_NO_SORTED_CHECK)
        log(f"block bytes {kind} {bb}")
        assert_parity(gpu_sort(s, a, kind, params=p), a, kind, ref)
