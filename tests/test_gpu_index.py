"""GPU index build (per-table stable radix sort + bucket offsets) against the
oracle's grouping: bit-exact sorted ids, distinct keys, offsets, counts."""
import numpy as np
import pytest

import oracle
from paper_2503_06737_amd import lsh
from gpu_util import dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _check(keys, id_base=0):
    ref = oracle.build_index(keys, id_base)
    idx = lsh.lsh_build_index(to_dev(keys), id_base=id_base)
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
