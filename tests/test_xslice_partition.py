"""CPU emulation of the x-slice family's row-block partition
(csrc/spmv_xslice.hip: k_xs_blocks, k_xs_split_count, k_xs_split_write and
the row -> block rule of k_xs_units), written out from the kernels'
formulas and checked on the benchmark's matrix shapes and edge cases:

* the row blocks cover the rows in order, each exactly once;
* no row block of several rows holds more than 4096 nonzeros (the slots a
  workgroup requests before it knows its count), none more than 4608 (its
  LDS slots), and every block holds fewer than 4096 cost units (nonzeros +
  rows) before its last row;
* the row -> block rule of the unit descriptors names the block that
  holds the row.

No GPU: this is host arithmetic on the kernels' formulas."""
import numpy as np
import pytest

import synth

DN = 4096
SPEC = 4096
DCAP = 4608


def partition(row_ptr):
    rp = row_ptr.astype(np.int64)
    n = rp.size - 1
    cost_row = rp[:-1] - rp[0] + np.arange(n)            # cost(i), strictly increasing
    total = int(rp[-1] - rp[0]) + n
    nbc = -(-total // DN)
    full = np.concatenate([cost_row, [total]])
    rbc = np.searchsorted(full, np.arange(nbc) * DN, side="left")  # first i with cost >= t*DN
    rbc = np.concatenate([rbc, [n]])
    a, b = rbc[:-1], rbc[1:]
    cnt = np.where((b > a + 1) & (rp[b] - rp[a] > SPEC), 2, 1)
    pos = np.concatenate([[0], np.cumsum(cnt)])
    nb = int(pos[-1])
    rb = np.empty(nb + 1, dtype=np.int64)
    rb[nb] = n
    rb[pos[:-1]] = a
    two = cnt == 2
    rb[pos[:-1][two] + 1] = b[two] - 1
    # row -> block, as the unit descriptors compute it
    tc = cost_row // DN
    t = pos[:-1][tc] + (np.arange(n) >= rb[pos[:-1][tc] + 1]).astype(np.int64)
    return rb, t


@pytest.mark.parametrize("n,seed,mean,max_len", [(1 << 18, 5, 16.0, 4096), (1 << 16, 502, 64.0, 4096),
                                                 (1 << 16, 501, 4.0, 4096), (5000, 7, 1.5, 40)])
def test_partition(n, seed, mean, max_len):
    m = synth.csr_matrix(n, seed, mean=mean, max_len=max_len)
    rp = m["row_ptr"].astype(np.int64)
    rb, t = partition(m["row_ptr"])
    assert rb[0] == 0 and rb[-1] == n and np.all(np.diff(rb) >= 0)
    elems = rp[rb[1:]] - rp[rb[:-1]]
    rows = np.diff(rb)
    assert elems.max() <= DCAP and np.all(elems[rows > 1] <= SPEC)
    nz = rows > 0
    last_len = rp[rb[1:][nz]] - rp[rb[1:][nz] - 1]
    assert np.all(elems[nz] - last_len + rows[nz] - 1 < DN)
    # every row in the block the rule names
    i = np.arange(n)
    assert np.all(rb[t] <= i) and np.all(i < rb[t + 1])


def test_split_blocks_on_long_rows():
    # rows of 3 nonzeros with some of 4000 to 4608: blocks ending in such a
    # row are split before it
    lens = np.full(5000, 3, dtype=np.int64)
    lens[[100, 1500, 1501, 3000, 4000, 4999]] = [4000, 4096, 4097, 2500, 4608, 4096]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    rb, t = partition(rp)
    elems = rp[rb[1:]].astype(np.int64) - rp[rb[:-1]]
    rows = np.diff(rb)
    assert elems.max() <= DCAP and np.all(elems[rows > 1] <= SPEC)
    for r in (100, 1500, 1501, 4000, 4999):
        assert rb[t[r] + 1] - rb[t[r]] >= 1 and t[r] == np.searchsorted(rb, r, side="right") - 1
