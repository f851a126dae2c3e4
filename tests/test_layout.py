"""Cell-blocked state layout of the C ABI (include/ssd.h): the binding's
pack_state / unpack_state against the index formula written out cell by
cell, on block-aligned and ragged element counts."""
import numpy as np
import pytest

from paper_1503_02198_amd.ssd import CB, pack_state, unpack_state


def _index(e, p, planes, E):
    b = e // CB
    nb = min(CB, E - CB * b)
    return b * CB * planes + p * nb + (e - CB * b)


@pytest.mark.parametrize("N,E", [(2, 1), (2, 63), (2, 64), (3, 65), (3, 130), (4, 200), (4, 256)])
def test_pack_matches_index_formula(N, E):
    Q = np.random.default_rng(N * 1000 + E).standard_normal((4, N, N, E)).astype(np.float32)
    P = 4 * N * N
    want = np.full(P * E, np.nan, np.float32)
    for e in range(E):
        for v in range(4):
            for j in range(N):
                for i in range(N):
                    want[_index(e, (v * N + j) * N + i, P, E)] = Q[v, j, i, e]
    assert not np.isnan(want).any()   # the formula is a bijection onto [0, 4 N^2 E)
    got = pack_state(Q)
    assert got.shape == (P * E,)
    assert np.array_equal(got, want)
    assert np.array_equal(unpack_state(got, N, E), Q)


def test_full_blocks_are_block_major():
    N, E = 2, 192
    Q = np.arange(4 * N * N * E, dtype=np.float32).reshape(4, N, N, E)
    q = pack_state(Q).reshape(E // CB, 4, N, N, CB)
    assert np.array_equal(q[1, 2, 1, 0], Q[2, 1, 0, CB:2 * CB])


def test_torch_tensors():
    import torch
    N, E = 3, 100
    Q = torch.randn(4, N, N, E, generator=torch.Generator().manual_seed(3))
    q = pack_state(Q)
    assert torch.equal(q, torch.from_numpy(pack_state(Q.numpy())))
    assert torch.equal(unpack_state(q, N, E), Q)


def test_wrong_sizes_are_rejected():
    with pytest.raises(ValueError):
        unpack_state(np.zeros(4 * 2 * 2 * 10 - 1, np.float32), 2, 10)
    with pytest.raises(ValueError):
        unpack_state(np.zeros((4, 40), np.float32), 2, 10)
    with pytest.raises(ValueError):
        pack_state(np.zeros(7, np.float32))
