"""GPU index build (per-table (key, id) order + bucket offsets) against the
oracle's grouping: bit-exact sorted ids, distinct keys, offsets, counts."""
import numpy as np
import pytest

import oracle
from paper_2503_06737_amd import lsh
from gpu_util import dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _check(keys, id_base=0):
    """Build on the current stream alone, then with the heavy-bucket kernels
    on a side stream; both indexes equal the oracle's."""
    import torch
    ref = oracle.build_index(keys, id_base)
    kd = to_dev(keys)
    for side in (None, torch.cuda.Stream(dev())):
        idx = lsh.lsh_build_index(kd, id_base=id_base, side_stream=side)
        assert idx.check() == (0, 0)
        sid, uk, of, nu = idx.arrays()
        L, n = keys.shape
        nu = to_host(nu)
        assert nu.tolist() == ref["nuniq"].tolist()
        sid = to_host(sid, np.uint32)
        assert (sid == ref["sorted_ids"]).all()
        uk, of = to_host(uk, np.uint64), to_host(of, np.uint32)
        for t in range(L):
            u = int(nu[t])
            assert (uk[t, :u] == ref["ukeys"][t, :u]).all()
            assert (of[t, :u + 1] == ref["offs"][t, :u + 1]).all()
    return idx


def _rng(seed):
    return np.random.default_rng(seed)


def test_random_keys_several_tiles_ragged():
    g = _rng(1)
    keys = g.integers(0, 2**63, (4, 4096 * 3 + 17), dtype=np.int64).astype(np.uint64) * np.uint64(2) \
        + g.integers(0, 2, (4, 4096 * 3 + 17)).astype(np.uint64)
    _check(keys)


def test_many_duplicates_and_id_base():
    g = _rng(2)
    small = g.integers(0, 300, (8, 20000)).astype(np.uint64)
    keys = small * np.uint64(0x9E3779B97F4A7C15)      # few distinct, spread over all bytes
    _check(keys, id_base=123456)


def test_srp_style_short_keys_skip_passes():
    g = _rng(3)
    keys = g.integers(0, 1 << 16, (16, 9000)).astype(np.uint64)
    _check(keys)


def test_all_equal_and_single_and_extremes():
    keys = np.full((3, 5000), 0xFFFFFFFFFFFFFFFF, np.uint64)
    keys[1] = 0
    keys[2] = 42
    _check(keys)
    _check(np.array([[7], [0]], np.uint64))
    g = _rng(4)
    k = g.integers(0, 2**63, (2, 3000), dtype=np.int64).astype(np.uint64)
    k[:, ::7] = np.uint64(0xFFFFFFFFFFFFFFFF)
    k[:, ::11] = 0
    _check(k)


def test_single_table_two_segments():
    """One table of at most 2048 keys has only two segments: the build's
    counters must still start at zero (they are cleared apart from the
    per-segment arrays)."""
    g = _rng(11)
    for n in (1, 5, 1000, 2048):
        keys = g.integers(0, 2**63, (1, n), dtype=np.int64).astype(np.uint64)
        keys[0, ::3] = keys[0, 0]
        _check(keys)


def test_head_look_back_over_many_tiles():
    """More than 64 head tiles (16K keys each) in one table: a tile's look-back
    crosses several windows of predecessors; many duplicates, ragged end."""
    g = _rng(12)
    n = 70 * 16384 + 123
    keys = g.integers(0, 200000, (1, n)).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    _check(keys, id_base=5)


@pytest.mark.parametrize("n", [300_000, 600_000])
def test_segment_digit_widths_8_and_9(n):
    """n that give an 8- and a 9-bit segment digit (the scatter's ballot count
    follows the width), two tables, digests with a heavy key."""
    g = _rng(13)
    keys = g.integers(0, 2**63, (2, n), dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        g.integers(0, 2, (2, n)).astype(np.uint64)
    keys[1, ::5] = keys[1, 7]
    _check(keys)


@pytest.mark.parametrize("nvary", [1, 8, 9])
def test_scattered_varying_bits(nvary):
    """Keys that differ only in nvary bits spread over the word (n = 300k:
    8-bit segment digits).  Up to 8 varying bits form the compacted digit
    (every segment one run of equal keys); 9 take the top-bits digit, whose
    segments then hold several keys (low varying bits outside the window)."""
    n, L = 300_000, 3
    g = _rng(70 + nvary)
    pos = np.sort(g.choice(64, nvary, replace=False))
    base = np.uint64(g.integers(0, 2**63)) & ~np.uint64(sum(1 << int(p) for p in pos))
    bits = g.integers(0, 2, (L, n, nvary), dtype=np.uint64)
    # skew: half of the points share one pattern (a heavy bucket)
    bits[:, : n // 2] = bits[:, :1]
    keys = np.full((L, n), base, np.uint64)
    for i, p in enumerate(pos):
        keys |= bits[:, :, i] << np.uint64(int(p))
    for t in range(L):
        g.shuffle(keys[t])
    _check(keys)


def test_empty_index():
    dev()
    import torch
    idx = lsh.lsh_build_index(torch.empty((3, 0), dtype=torch.int64, device="cuda"))
    _, _, of, nu = idx.arrays()
    assert to_host(nu).tolist() == [0, 0, 0] and to_host(of).tolist() == [[0], [0], [0]]


def test_key_ld_strided_input():
    """Keys read from a [L][key_ld] buffer with key_ld > n."""
    dev()
    g = _rng(5)
    full = g.integers(0, 1000, (4, 7000)).astype(np.uint64) * np.uint64(0x100000001B3)
    n = 6000
    ref = oracle.build_index(np.ascontiguousarray(full[:, :n]))
    t = to_dev(full)[:, :n]
    idx = lsh.lsh_build_index(t)
    sid = to_host(idx.arrays()[0], np.uint32)
    assert (sid == ref["sorted_ids"]).all()


# ---- segments larger than one LDS sort (8192 keys) and the prefix check

def test_heavy_bucket_spans_several_tiles():
    """40% of a table share one key: its segment (top varying byte) exceeds the
    LDS sort and is ordered by the segmented global pass; other tables mix
    sizes so both parities of the pass count occur."""
    g = _rng(6)
    n = 40000
    keys = g.integers(0, 2**63, (3, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    heavy = g.random((3, n)) < 0.4
    keys[0][heavy[0]] = np.uint64(0x8123456789ABCDEF)
    # table 1: heavy key differs from its segment-mates only in the low 16 bits
    keys[1][heavy[1]] = np.uint64(0x7700000000001234)
    keys[1][::97] = np.uint64(0x7700000000000000) + g.integers(0, 1 << 16, keys[1][::97].size).astype(np.uint64)
    # table 2: two heavy keys in the same top byte
    keys[2][heavy[2]] = np.uint64(0x5500000000000001)
    keys[2][heavy[2] & (g.random(n) < 0.5)] = np.uint64(0x55FF000000000001)
    _check(keys, id_base=1000)


def test_all_equal_large_and_segment_size_boundary():
    n = 20000
    keys = np.full((2, n), 0x0123456789ABCDEF, np.uint64)
    # table 1: exactly 8192 keys in one segment, 8193 in another, rest spread
    g = _rng(7)
    k1 = g.integers(0, 2**63, n, dtype=np.int64).astype(np.uint64)
    top = k1 >> np.uint64(56)
    k1[top == 0x11] ^= np.uint64(0x0100000000000000)   # empty segments 0x11 and 0x22
    k1[top == 0x22] ^= np.uint64(0x0100000000000000)
    k1[:8192] = (k1[:8192] & np.uint64(0x00FFFFFFFFFFFFFF)) | np.uint64(0x1100000000000000)
    k1[8192:8192 + 8193] = (k1[8192:8192 + 8193] & np.uint64(0x00FFFFFFFFFFFFFF)) | np.uint64(0x2200000000000000)
    keys[1] = k1
    _check(keys)


def test_segment_sizes_at_the_workgroup_boundaries():
    """Segments (top 5 varying bits for n = 40000) of exactly 2048 and 2049
    keys (the two LDS sort sizes) and 4096 / 4097 (the LDS sort and the big
    path), with duplicates inside them; the rest spread over other digits."""
    g = _rng(10)
    n = 40000
    keys = g.integers(0, 2**63, (2, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    top = keys >> np.uint64(59)
    for d in (3, 7, 11, 19):
        keys[top == d] ^= np.uint64(1) << np.uint64(59)    # keep these digits empty
    low = np.uint64((1 << 59) - 1)
    start = 0
    for d, size in ((3, 2048), (7, 2049), (11, 4096), (19, 4097)):
        sl = slice(start, start + size)
        keys[:, sl] = (keys[:, sl] & low) | (np.uint64(d) << np.uint64(59))
        keys[:, start + 5:start + size:9] = keys[:, start:start + 1]   # a repeated key
        start += size
    keys[1] = keys[1, g.permutation(n)]
    _check(keys, id_base=77)


def test_skewed_short_keys_big_segments():
    """16-bit keys from a few values (clustered SRP codes): segments by the
    high byte are far larger than 8192 and differ only in the low byte."""
    g = _rng(8)
    vals = g.integers(0, 1 << 16, 12).astype(np.uint64)
    vals[1] = (vals[0] & np.uint64(0xFF00)) | np.uint64(0x3)
    keys = vals[g.integers(0, vals.size, (4, 50000))]
    _check(keys)


def test_prefix_check_falls_back_to_every_chunk():
    """Distinct keys that agree on bits 24..63 inside one small segment: the
    four-chunk sort alone would leave them in id order, the adjacent-pair
    check must trigger the full sort."""
    g = _rng(9)
    n = 6000
    keys = g.integers(0, 2**63, (2, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    for t in range(2):
        src = g.integers(0, n, 800)
        dst = g.integers(0, n, 800)
        low = g.integers(1, 1 << 24, 800).astype(np.uint64)
        keys[t, dst] = keys[t, src] ^ low              # siblings: same bits 24..63
        keys[t, dst[:100]] = keys[t, src[:100]]        # and some exact duplicates
    _check(keys)


@pytest.mark.slow
def test_sparse_image_rows_index_from_oracle_keys():
    """Keys of the image-like workload (heavy all-zero-code bucket per table),
    computed by the oracle, indexed on the GPU: every table bit-exact."""
    from paper_2503_06737_amd import synth
    wl = synth.C2
    n, K, L = 120000, wl.K, 16
    x = wl.points(n).astype(np.float64)
    h, s = synth.cs_state(wl.d, K * L, wl.seed + 1)
    b = synth.shifts(K * L, wl.w, wl.seed + 1)
    keys = oracle.hash_points(x, oracle.E2LSH, K, L, kind="cs", w=wl.w, b=b, h=h, s=s)["keys"]
    _check(keys)


def test_builds_on_two_streams_and_threads_read_back_on_their_own_stream():
    """Heavy buckets send segments to the big-segment kernels, which run on
    the side stream the build is given.  Two host threads build at once, each
    on a non-default stream with a side stream of its own; each reads its
    index back with copies enqueued on its main stream only (no device-wide
    synchronisation), so the copies see the side stream's results only if
    the main stream waits for them.  Both indexes equal the oracle's on every
    repetition."""
    import threading
    import torch
    g = _rng(21)
    n = 60000
    sets = []
    for i in range(2):
        keys = g.integers(0, 2**63, (4, n), dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
        heavy = g.random((4, n)) < 0.3
        keys[heavy] = np.uint64(0x8123456789ABCDEF) + np.uint64(2 * i)
        keys[1][g.random(n) < 0.2] = np.uint64(0x55) << np.uint64(56)
        sets.append(keys)
    refs = [oracle.build_index(k, 7) for k in sets]
    d = dev()
    kd = [to_dev(k) for k in sets]
    torch.cuda.synchronize()
    got = [[], []]
    errs = []

    def run(i):
        try:
            st, side = torch.cuda.Stream(d), torch.cuda.Stream(d)
            with torch.cuda.stream(st):
                for _ in range(3):
                    idx = lsh.lsh_build_index(kd[i], id_base=7, side_stream=side)
                    sid, uk, of, nu = idx.arrays()
                    got[i].append((sid.to("cpu"), uk.to("cpu"), of.to("cpu"), nu.to("cpu"),
                                   idx.check()))
        except Exception as e:  # surfaced in the main thread
            errs.append(e)

    ths = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errs, errs
    for i in range(2):
        ref = refs[i]
        assert len(got[i]) == 3
        for sid, uk, of, nu, chk in got[i]:
            assert chk == (0, 0)
            nu = nu.numpy()
            assert nu.tolist() == ref["nuniq"].tolist()
            assert (sid.numpy().view(np.uint32) == ref["sorted_ids"]).all()
            uk, of = uk.numpy().view(np.uint64), of.numpy().view(np.uint32)
            for t in range(4):
                u = int(nu[t])
                assert (uk[t, :u] == ref["ukeys"][t, :u]).all()
                assert (of[t, :u + 1] == ref["offs"][t, :u + 1]).all()


def test_side_stream_equal_to_the_main_stream():
    """A side stream that is the main stream itself forks nothing: the build
    runs on that stream alone and equals the oracle's (heavy buckets, so the
    big-segment kernels run)."""
    import torch
    g = _rng(23)
    n = 30000
    keys = g.integers(0, 2**63, (3, n), dtype=np.int64).astype(np.uint64) * np.uint64(2)
    keys[g.random((3, n)) < 0.35] = np.uint64(0x9123456789ABCDEF)
    ref = oracle.build_index(keys, 0)
    idx = lsh.lsh_build_index(to_dev(keys), side_stream=torch.cuda.current_stream())
    assert idx.check() == (0, 0)
    sid, uk, of, nu = idx.arrays()
    nu = to_host(nu)
    assert nu.tolist() == ref["nuniq"].tolist()
    assert (to_host(sid, np.uint32) == ref["sorted_ids"]).all()
    uk, of = to_host(uk, np.uint64), to_host(of, np.uint32)
    for t in range(3):
        u = int(nu[t])
        assert (uk[t, :u] == ref["ukeys"][t, :u]).all()
        assert (of[t, :u + 1] == ref["offs"][t, :u + 1]).all()
