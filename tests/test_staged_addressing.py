"""CPU emulation of the staged level-0 addressing of the register z-march
with three or four fused sweeps (csrc/zmarch.h, tb_column with STAGE, and
the wave selection in csrc/jacobi.hip and csrc/batch.hip).

The index formulas of the kernel are written out here and checked over
whole launches, including 74-plane z-chunks and boundary waves:

* every 16-byte global->LDS piece reads inside the grid (clamped
  coordinates) and lands inside its wave's buffer;
* every level-0 value, and every x-neighbour level 1 takes (four sweeps)
  or strip-edge value (fewer), that the march reads back from LDS comes
  from the intended grid point whenever that point lies inside the grid
  (points outside are zeroed by the kernel, so any clamped piece there is
  harmless);
* a plane buffer is refilled only after the plane it held has been read
  (two buffers, plane kp in buffer kp & 1, refill of plane k+2 after the
  reads of iteration k);
* the per-wave staging slots of the batched three-sweep kernel (one fixed
  stride, the widest tile's) are disjoint and inside the block's LDS area
  for every (T, R) it runs.

No GPU: this is host arithmetic on the kernel's formulas."""
import pytest

ROW_B = 68 * 8  # bytes of one staged row (68 doubles from the even x0)


def nl(T, R, level):
    return R + 2 * (T - level)


def stage_wave_bytes(T, R):
    return 2 * ((nl(T, R, 0) * 34 + 63) // 64) * 1024


def pieces(T, R, nx, ny, i0, j0):
    """(global element (jr, xr) of each lane's piece, LDS byte offset) per
    copy instruction p and lane, as the kernel computes them."""
    n0 = nl(T, R, 0)
    k_pieces = n0 * 34
    k_copies = (k_pieces + 63) // 64
    x0 = i0 - 2 - (i0 & 1)
    out = []
    for p in range(k_copies):
        for lane in range(64):
            g = p * 64 + lane
            r = min(g // 34, n0 - 1)
            c = min(g - r * 34, 33)
            jr = min(max(j0 - T + r, 0), ny - 1)
            xr = min(max(x0 + 2 * c, 0), nx - 2)
            lds = p * 1024 + lane * 16  # copy p of a wave writes 64 lanes x 16 bytes
            out.append((r, c, jr, xr, lds))
    return out, k_copies * 1024, x0


def check_wave(T, R, nx, ny, nz, i0, j0, k0, k1):
    n0 = nl(T, R, 0)
    plist, kbuf, x0 = pieces(T, R, nx, ny, i0, j0)
    # LDS byte -> grid element (row, x) that the piece put there
    lds_map = {}
    for r, c, jr, xr, lds in plist:
        assert 0 <= jr < ny and 0 <= xr and xr + 1 < nx  # the 16 bytes read lie in the row
        assert 0 <= lds and lds + 16 <= kbuf              # inside one plane buffer
        lds_map[lds] = (jr, xr)
        lds_map[lds + 8] = (jr, xr + 1)
    sh = i0 - x0
    assert sh in (2, 3)
    ka = k0 - T + 1
    kend = k1 + T - 2

    def staged_plane(kp):
        return min(max(kp, 0), nz - 1)

    def read(kp, q, off, x_want, j_want):
        """Value read at byte q * ROW_B + off of plane kp's buffer: if the
        point is inside the grid it must be the intended element."""
        if not (0 <= kp < nz and 0 <= j_want < ny and 0 <= x_want < nx):
            return  # zeroed by the kernel
        byte = q * ROW_B + off
        assert byte + 8 <= kbuf
        assert byte in lds_map, (q, off)
        assert staged_plane(kp) == kp
        assert lds_map[byte] == (j_want, x_want), (kp, q, off, lds_map[byte], (j_want, x_want))

    # buffer b holds plane `held[b]`; planes read in iteration k: k+1 (level
    # 0) and k (level 1's x-neighbours or the strip edges); refilled after
    # those reads: plane k+2 into (k+2) & 1
    held = {ka & 1: ka, (ka + 1) & 1: ka + 1}
    for k in range(ka, kend + 1):
        assert held[(k + 1) & 1] == k + 1 and held[k & 1] == k
        for lane in range(64):
            i = i0 + lane
            xo = (lane + sh) * 8
            for q in range(n0):
                read(k + 1, q, xo, i, j0 - T + q)
            if T >= 4:
                # level 1's x-neighbours: the lane's x-1 and x+1 in plane k's row
                for q in range(nl(T, R, 1)):
                    read(k, q + 1, xo - 8, i - 1, j0 - (T - 1) + q)
                    read(k, q + 1, xo + 8, i + 1, j0 - (T - 1) + q)
            else:
                # the strip edges: x = i0-1 on lane 0, x = i0+64 on lane 63
                eo = (sh - 1) * 8 if lane == 0 else (64 + sh) * 8 if lane == 63 else xo
                ie = i0 - 1 if lane == 0 else i0 + 64 if lane == 63 else i
                for q in range(nl(T, R, 1)):
                    read(k, q + 1, eo, ie, j0 - (T - 1) + q)
        if k < kend:
            held[(k + 2) & 1] = k + 2  # plane k's buffer, read above


def staged_waves_grid(T, R, nx, ny, nz, bz, waves=4):
    """Waves of the per-grid kernel that take the staged march, with their
    (i0, j0, k0, k1), following the selection in jacobi.hip."""
    W = 66 - 2 * T
    nbx = -(-nx // W)
    nby = -(-ny // (waves * R))
    k_edges = (T == 4 and R <= 4) or (T == 3 and R <= 6)
    for kb in range(-(-nz // bz)):
        for bj in range(nby):
            for bi in range(nbx):
                for w in range(waves):
                    j0 = (bj * waves + w) * R
                    if j0 >= ny:
                        continue
                    i0 = W * bi - (T - 1)
                    x0 = i0 - 2 - (i0 & 1)
                    inner = i0 >= 1 and i0 + 64 < nx and j0 >= T and j0 + R + T <= ny
                    fits = nx >= 2 and nx * ny * 8 < 2 ** 32 and (nx % 2 == 0 or x0 + 68 <= nx)
                    if (fits and inner and x0 >= 0 and x0 + 68 <= nx) or (k_edges and fits):
                        yield i0, j0, kb * bz, min(nz, kb * bz + bz)


@pytest.mark.parametrize("T,R,shape,bz", [
    (4, 4, (130, 37, 160), 74),   # 74-plane z-chunks: one whole, one ragged (86 planes)
    (4, 4, (127, 20, 80), 74),    # odd nx: only waves whose 68 columns fit stage
    (4, 1, (64, 9, 10), 3),
    (3, 4, (201, 33, 50), 22),
    (3, 1, (70, 5, 9), 1),
    (3, 6, (96, 50, 30), 16),
    (4, 5, (150, 48, 30), 74),    # more rows than the boundary waves stage: inner waves only
    (4, 4, (130, 40, 9), 1),      # one-plane chunks (the device-filling chunk of small grids)
    (4, 4, (130, 40, 9), 2),      # and two-plane chunks with a ragged last one
    (3, 4, (130, 40, 7), 3),
    (3, 2, (130, 21, 11), 2),     # two rows per wave, filled chunks
])
def test_per_grid_staged_addressing(T, R, shape, bz):
    nx, ny, nz = shape
    n = 0
    for i0, j0, k0, k1 in staged_waves_grid(T, R, nx, ny, nz, bz):
        check_wave(T, R, nx, ny, nz, i0, j0, k0, k1)
        n += 1
    assert n > 0


def test_batched_slots_disjoint_and_inside():
    # the three-sweep batch kernel runs staged marches of (T, R) in
    # {2, 3} x {1, 2, 4} with one fixed per-wave stride: the widest tile's
    stride = stage_wave_bytes(3, 4)
    block = 4 * stage_wave_bytes(3, 4)
    for T in (2, 3):
        for R in (1, 2, 4):
            need = stage_wave_bytes(T, R)
            assert need <= stride
            spans = [(w * stride, w * stride + need) for w in range(4)]
            for a, b in zip(spans, spans[1:]):
                assert a[1] <= b[0]
            assert spans[-1][1] <= block
            # and the pieces of any wave land inside its own span
            plist, kbuf, _ = pieces(T, R, 500, 300, 61, 17)
            assert 2 * kbuf == need
            assert all(lds + 16 <= kbuf for *_, lds in plist)
