"""Pins of the CPU oracle against facts fixed outside it: published
known-answer values, hand-evaluated formulas from the paper, library
routines (numpy sort, bisect, Python's bytes ordering), closed forms of the
input distributions, and brute force on tiny inputs."""
import bisect
import itertools
import math
import os
from collections import Counter

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_splitmix64_known_answers():
    for row in _lines("splitmix64_kat.txt"):
        state, outs = int(row[0], 0), [int(x, 16) for x in row[1:]]
        assert oracle.splitmix64(state, len(outs)) == outs
        # the input generators implement the same published generator separately
        assert [int(x) for x in synth.stream(state, len(outs))] == outs


def test_mulhi64_exact():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = int(rng.integers(0, 2**63)) * 2 + 1, int(rng.integers(0, 2**63))
        assert oracle.mulhi64(a, b) == (a * b) >> 64


def test_task_rules_hand_values():
    for name, n, v in _lines("task_rules.txt"):
        n, v = int(n), int(v)
        if name == "alpha":
            assert oracle.alpha(n) == v, n
        else:
            assert oracle.adaptive_k(n, 256, 16) == v, n


def test_adaptive_k_against_real_valued_formula():
    # The printed formula evaluated in floating point at sizes where no
    # rounding decision is close to an integer boundary.
    rng = np.random.default_rng(2)
    k, n0 = 256, 16
    for n in rng.integers(17, 1 << 22, size=3000).tolist():
        x = math.log2(n / n0)
        if k * n0 < n < k * k * n0:
            t = (x + 1) / 2
            if abs(t - round(t)) < 1e-9:
                continue
            want = 2 ** math.ceil(t)
        elif n0 < n <= k * n0:
            if abs(x - round(x)) < 1e-9:
                continue
            want = 2 ** math.ceil(x)
        else:
            want = k
        assert oracle.adaptive_k(n, k, n0) == max(2, min(k, want)), n


KINDS = ["u32", "u64", "f64", "pair", "rec100", "quartet"]


def _keys(a, kind):
    """Sort keys as Python objects whose natural order is the key order."""
    if kind == "u32" or kind == "u64":
        return [int(x) for x in a]
    if kind == "f64":
        return [float(x) for x in a]
    if kind == "pair":
        return [int(x) for x in a[:, 0]]
    if kind == "quartet":
        return [tuple(int(v) for v in r[:3]) for r in a]
    return [bytes(r[:10]) for r in a]


def _multiset(a, kind):
    if a.ndim == 1:
        return Counter(a.tobytes()[i * a.itemsize:(i + 1) * a.itemsize] for i in range(a.shape[0]))
    return Counter(bytes(r.tobytes()) for r in a)


def _gen(kind, dist, n, seed):
    if kind == "f64":
        return synth.gen_f64("uniform" if dist not in ("exponential",) else dist, n, seed)
    if kind == "rec100":
        return synth.gen_rec100("rootdup" if dist == "rootdup" else "uniform", n, seed)
    if kind == "quartet":
        return synth.gen_quartet(dist, n, seed)
    if kind == "u32" and dist == "twodup" or kind == "u32" and dist == "eightdup":
        return synth.gen_u32(dist, n, seed)
    return synth.generate(kind, dist, n, seed)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000, 65536])
def test_sort_matches_library_sort(kind, n):
    for dist in ("uniform", "rootdup", "twodup"):
        a = _gen(kind, dist, n, 11 + n)
        s = oracle.sort(a, kind)
        k = _keys(s, kind)
        assert k == sorted(_keys(a, kind))          # library sort of the keys
        assert _multiset(s, kind) == _multiset(a, kind)
        if kind in ("u32", "u64", "f64"):
            assert np.array_equal(s, np.sort(a, kind="stable"))


def _oracle_sort_segments(arr, kind, n):
    """The oracle run in place on every consecutive n-element segment."""
    import ctypes
    L, D = oracle.lib(), oracle.ELEM_BYTES[kind]
    base = arr.ctypes.data
    for off in range(0, arr.shape[0], n):
        assert L.oracle_sort(ctypes.c_void_p(base + off * D), n, oracle.TYPES[kind]) == 0
    return arr


def _key_list(a, kind):
    """Keys as comparable Python values: integers (f64: the bit pattern,
    whose order is checked against the hand-ordered list) or bytes."""
    if kind == "f64":
        return a.view(np.uint64).tolist()
    if kind == "pair":
        return a[:, 0].tolist()
    if kind == "rec100":
        return [bytes(r[:10]) for r in a]
    if kind == "quartet":
        return [tuple(int(v) for v in r[:3]) for r in a]
    return a.tolist()


@pytest.mark.parametrize("kind", KINDS)
def test_sort_brute_force_tiny(kind):
    """Every permutation of n <= 8 distinct keys and every sequence of n <= 8
    keys over three values (tests/bruteforce_cases.py).  A permutation must
    come out as the keys in their listed (hand-ordered) order; a sequence
    must come out non-decreasing in the listed order with its multiset
    unchanged; pair values and record payloads must still name an input
    element with the same key."""
    import bruteforce_cases as bc
    vals = bc.key_values(kind)
    if kind in ("u32", "u64", "pair", "rec100", "quartet"):
        assert vals == sorted(vals)          # library order agrees with the listed order
    else:                                    # the listed doubles follow the golden totalOrder list
        gold = [int(r[0], 16) for r in _lines("f64_total_order.txt")]
        assert [gold.index(v) for v in vals] == sorted(gold.index(v) for v in vals)
    tri = bc.tri_values(kind)
    rank = {v: i for i, v in enumerate(tri)}
    for n in range(1, bc.NMAX + 1):
        inp = bc.build(kind, bc.permutation_seqs(kind, n))
        out = _oracle_sort_segments(inp.copy(), kind, n)
        want = vals[:n]
        keys = _key_list(out, kind)
        assert all(keys[o:o + n] == want for o in range(0, len(keys), n)), (kind, n)
        if kind in ("pair", "rec100", "quartet"):
            ix = (out[:, 1] if kind == "pair" else out[:, 3] if kind == "quartet"
                  else out[:, 10:18].copy().view("<u8")[:, 0]).astype(np.int64)
            assert np.array_equal(np.sort(ix), np.arange(inp.shape[0]))
            assert np.array_equal(out, inp[ix])            # whole records moved intact
            assert all(set(ix[o:o + n] // n) == {o // n} for o in range(0, len(ix), n))
        seqs = bc.ternary_seqs(kind, n)
        inp = bc.build(kind, seqs)
        out = _oracle_sort_segments(inp.copy(), kind, n)
        keys = _key_list(out, kind)
        for i, sq in enumerate(seqs):
            got = keys[i * n:(i + 1) * n]
            r = [rank[x] for x in got]
            assert r == sorted(r) and Counter(got) == Counter(sq), (kind, sq, got)


def test_sort_brute_force_multiset_u32():
    """Sequences over {0, 1, 2} against Python's sorted (library)."""
    for n in range(0, 8):
        for seq in itertools.product(range(3), repeat=n):
            a = np.array(seq, dtype=np.uint32)
            assert oracle.sort(a, "u32").tolist() == sorted(seq)


def test_pair_sort_values_are_indices():
    a = synth.gen_pair("rootdup", 5000, 3)
    s = oracle.sort(a, "pair")
    assert sorted(s[:, 1].tolist()) == list(range(5000))
    assert np.array_equal(a[s[:, 1].astype(np.int64), 0], s[:, 0])


def test_rec100_order_is_unsigned_bytes():
    a = synth.gen_rec100("uniform", 3000, 5)
    a[::7, 0] = 0xFF      # bytes >= 0x80 must sort after small ones
    a[1::7, 0:10] = a[0, 0:10]
    s = oracle.sort(a, "rec100")
    assert [bytes(r[:10]) for r in s] == sorted(bytes(r[:10]) for r in a)
    assert _multiset(s, "rec100") == _multiset(a, "rec100")


def test_f64_total_order_golden():
    want = [int(r[0], 16) for r in _lines("f64_total_order.txt")]
    bits = np.array(want, dtype=np.uint64)
    rng = np.random.default_rng(4)
    for _ in range(20):
        shuffled = bits[rng.permutation(bits.size)].view(np.float64)
        s = oracle.sort(shuffled.copy(), "f64")
        assert s.view(np.uint64).tolist() == want


@pytest.mark.parametrize("n", [1000, 4096, 65536])
def test_closed_forms_of_distributions(n):
    assert np.array_equal(oracle.sort(synth.gen_u64("almostsorted", n, 9), "u64"),
                          np.arange(n, dtype=np.uint64))
    assert not oracle.sort(synth.gen_u64("zero", n, 9), "u64").any()
    m = math.isqrt(n)
    rd = oracle.sort(synth.gen_u64("rootdup", n, 9), "u64")
    want = np.repeat(np.arange(m, dtype=np.uint64), [(n - 1 - v) // m + 1 for v in range(m)])
    assert np.array_equal(rd, want)
    for dist in ("twodup", "eightdup", "exponential"):
        a = synth.gen_u64(dist, n, 9)
        cnt = np.bincount(a.astype(np.int64))                    # counting sort
        assert np.array_equal(oracle.sort(a, "u64"),
                              np.repeat(np.arange(cnt.size, dtype=np.uint64), cnt))
    s = synth.gen_u64("sorted", n, 9)
    assert np.array_equal(oracle.sort(s[::-1].copy(), "u64"), s)


def _classify_pins(keys, spl, K, kind):
    """Pin oracle_classify with bisect (library) and the equality-bucket
    properties: odd bucket 2i+1 holds exactly the keys equal to s_i, even
    bucket 2i the keys strictly between s_{i-1} and s_i, bucket 2K-1 the keys
    above every splitter, bucket 2K-2 nothing."""
    sk = [int(x) for x in spl[:K - 1]]
    for e in keys:
        e_arr = np.array([e], dtype=spl.dtype)
        i = bisect.bisect_left(sk, int(e))
        assert oracle.classify(e_arr, kind, spl, K, False) == i
        b = oracle.classify(e_arr, kind, spl, K, True)
        if b % 2 == 1 and b < 2 * K - 1:
            assert int(e) == sk[b // 2]
        elif b == 2 * K - 1:
            assert int(e) > sk[-1]
        else:
            assert b != 2 * K - 2
            j = b // 2
            assert (j == 0 or sk[j - 1] < int(e)) and int(e) < sk[j]


def test_classify_exhaustive_small_domain():
    rng = np.random.default_rng(5)
    for K in (2, 4, 8):
        for _ in range(60):
            u = int(rng.integers(1, K))              # distinct splitters, padded
            vals = np.sort(rng.choice(16, size=u, replace=False)).astype(np.uint32)
            spl = np.concatenate([vals, np.full(K - u, vals[-1], dtype=np.uint32)])
            _classify_pins(range(16), spl, K, "u32")


def test_classify_monotone_and_histogram():
    a = synth.gen_u64("twodup", 1 << 14, 2)
    st = oracle.sample_step(a, "u64", seed=7, k=64)
    spl, K = st["splitters"], st["K"]
    for eq in (False, True):
        h = oracle.histogram(a, "u64", spl, K, eq)
        keys = np.sort(a)
        bk = [oracle.classify(np.array([x], dtype=np.uint64), "u64", spl, K, eq) for x in keys[::37]]
        assert bk == sorted(bk)
        if not eq:
            idx = np.searchsorted(spl[:K - 1], a, side="left")      # library
            assert np.array_equal(h, np.bincount(idx, minlength=K).astype(np.uint64))
        assert int(h.sum()) == a.size


@pytest.mark.parametrize("dist", ["uniform", "rootdup", "eightdup", "zero"])
def test_sample_step_definition(dist):
    n, seed, l = 1 << 16, 99, 0
    a = synth.gen_u64(dist, n, 4)
    st = oracle.sample_step(a, "u64", l=l, n=n, seed=seed)
    alpha, kp = st["alpha"], st["k_prime"]
    assert (alpha, kp) == (3, 128)                # hand values: 16/5 -> 3; 2^16 -> 128
    assert st["m"] == alpha * kp
    # Sample positions recomputed with the generator module's own SplitMix64
    # and Python big integers.
    ts_state = (seed ^ ((l * 0x9E3779B97F4A7C15) & (2**64 - 1)) ^ (0 << 56))
    _, tseed = synth.splitmix64_scalar(ts_state)
    assert oracle.task_seed(seed, l, 0) == tseed
    xs = synth.stream(tseed, st["m"])
    pos = [l + ((int(x) * n) >> 64) for x in xs]
    assert np.array_equal(st["sample"], np.sort(a[pos]))
    pick = [st["sample"][(i + 1) * alpha - 1] for i in range(kp - 1)]
    distinct = sorted(set(int(x) for x in pick))
    assert st["u"] == len(distinct)
    assert st["eq"] == (len(distinct) < kp - 1)
    K = st["K"]
    assert K >= st["u"] + 1 and K // 2 < st["u"] + 1 and K & (K - 1) == 0
    assert [int(x) for x in st["splitters"]] == distinct + [distinct[-1]] * (K - len(distinct))


def test_check_partition_detects_planted_mistake():
    a = synth.gen_u64("uniform", 1 << 12, 8)
    st = oracle.sample_step(a, "u64", seed=1, k=16)
    spl, K = st["splitters"], st["K"]
    b = np.array([oracle.classify(np.array([x], dtype=np.uint64), "u64", spl, K, False) for x in a])
    order = np.argsort(b, kind="stable")
    part = a[order]
    starts = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=K))]).astype(np.uint64)
    assert oracle.check_partition(part, "u64", spl, K, False, starts) is None
    bad = part.copy()
    i, j = int(starts[1]) - 1, int(starts[2])       # swap across a boundary
    bad[i], bad[j] = bad[j], bad[i]
    assert oracle.check_partition(bad, "u64", spl, K, False, starts) in (i, j)


def test_radix_digit_info_hand_values():
    a = np.array([0x1234, 0x1200, 0x1210], dtype=np.uint64)       # xor 0x34: h = 5
    assert oracle.radix_digit_info(a, "u64") == {"shift": 0, "width": 6, "all_equal": False}
    rd = synth.gen_u64("rootdup", 1 << 20, 0)                     # 0..1023: h = 9
    assert oracle.radix_digit_info(rd, "u64") == {"shift": 2, "width": 8, "all_equal": False}
    assert oracle.radix_digit_info(np.full(5, 7, dtype=np.uint32), "u32")["all_equal"]
    h = oracle.radix_histogram(rd, "u64", 2, 8)
    assert np.array_equal(h, np.full(256, 4096, dtype=np.uint64))


def test_radix_key_of_doubles():
    """The unsigned image of a double used by the radix variant keeps IEEE
    754 totalOrder.  Hand values: +0.0 maps to 0x8000000000000000 and -0.0 to
    0x7FFFFFFFFFFFFFFF, so their highest differing bit is 63 and the top
    digit is 0x80 and 0x7F; +inf (0xFFF0...) and +NaN (0xFFF8...) differ
    first at bit 51; -inf maps to 0x000F... and -1.0 to 0x400F..., first
    differing at bit 62.  Order: for each consecutive pair x < y of the
    golden totalOrder list, the array [x, x, y] puts both x into digit 0 of
    the one-bit digit at their highest differing bit."""
    f = lambda *bits: np.array(bits, dtype=np.uint64).view(np.float64)
    z = f(0x0000000000000000, 0x8000000000000000)
    assert oracle.radix_digit_info(z, "f64") == {"shift": 56, "width": 8, "all_equal": False}
    h = oracle.radix_histogram(z, "f64", 56, 8)
    assert h[0x80] == 1 and h[0x7F] == 1 and int(h.sum()) == 2
    inf_nan = f(0x7FF0000000000000, 0x7FF8000000000000)
    assert oracle.radix_digit_info(inf_nan, "f64") == {"shift": 44, "width": 8, "all_equal": False}
    h = oracle.radix_histogram(inf_nan, "f64", 44, 8)
    assert h[0x00] == 1 and h[0x80] == 1
    neg = f(0xFFF0000000000000, 0xBFF0000000000000)            # -inf, -1.0
    assert oracle.radix_digit_info(neg, "f64") == {"shift": 55, "width": 8, "all_equal": False}
    h = oracle.radix_histogram(neg, "f64", 55, 8)
    assert h[0x00] == 1 and h[0x80] == 1
    assert oracle.radix_digit_info(f(0x7FF8000000000001, 0x7FF8000000000001), "f64")["all_equal"]
    gold = [int(r[0], 16) for r in _lines("f64_total_order.txt")]
    for x, y in zip(gold, gold[1:]):
        a = f(x, x, y)
        d = oracle.radix_digit_info(a, "f64")
        top = d["shift"] + d["width"] - 1
        assert oracle.radix_histogram(a, "f64", top, 1).tolist() == [2, 1], (hex(x), hex(y))


def test_count_less_matches_searchsorted():
    a = synth.gen_u64("rootdup", 10000, 1)
    s = np.sort(a)
    for v in (0, 5, 50, 99, 1000):
        x = np.array([v], dtype=np.uint64)
        assert oracle.count_less(a, "u64", x) == int(np.searchsorted(s, v, "left"))
        assert oracle.count_less(a, "u64", x, True) == int(np.searchsorted(s, v, "right"))


def test_quartet_order_is_lexicographic():
    """Algorithm 3: a decides, then b, then c; the fourth word is payload."""
    rng = np.random.default_rng(12)
    a = rng.integers(0, 4, size=(4000, 4), dtype=np.uint64)   # many ties in every word
    a[:, 3] = np.arange(4000, dtype=np.uint64)
    s = oracle.sort(a, "quartet")
    assert [tuple(r[:3]) for r in s.tolist()] == sorted(tuple(r[:3]) for r in a.tolist())
    assert np.array_equal(a[s[:, 3].astype(np.int64)], s)
    big = np.array([[1, 0, 0, 0], [0, 0xFFFFFFFFFFFFFFFF, 0, 1], [0, 0, 0xFFFFFFFFFFFFFFFF, 2]], dtype=np.uint64)
    assert oracle.sort(big, "quartet")[:, 3].tolist() == [2, 1, 0]
