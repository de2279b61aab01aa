"""Host logic of AO_VF_FILL_Z: the planes per block a register z-march
launch takes, queried through the C ABI with a given number of resident
workgroups (no device needed), against the rule written out by brute force:
the chunk length b <= bz that minimises ceil(blocks(b) / resident) * (b +
2(T-1)), ties to the longer chunk."""
import itertools

import pytest

import paper_2303_08873_amd as ao

G = ao.AO_TARGET_GPU
cd = lambda a, b: -(-a // b)  # noqa: E731

# (family, fused sweeps T, stored columns per 64-lane strip)
FAMS = [(ao.FAM_JACOBI_ZREG, 1, 64), (ao.FAM_JACOBI_ZREG_T2, 2, 62),
        (ao.FAM_JACOBI_ZREG_T3, 3, 60), (ao.FAM_JACOBI_ZREG_T4, 4, 58)]


def rule(nx, ny, nz, T, width, R, bz, resident):
    cols = cd(nx, width) * cd(ny, 4 * R)
    best = None
    for b in range(1, min(bz, nz) + 1):
        cost = cd(cols * cd(nz, b), resident) * (b + 2 * (T - 1))
        if best is None or cost <= best[0]:
            best = (cost, b)
    return best[1]


@pytest.mark.parametrize("fam,T,width", FAMS)
def test_planes_follow_the_rule(fam, T, width):
    R = 4
    flags = ao.AO_VF_FILL_Z | (ao.AO_VF_STAGED if T >= 3 else 0)
    for (nx, ny, nz), bz, res in itertools.product(
            [(16, 16, 16), (64, 64, 64), (100, 37, 250), (256, 256, 256), (512, 512, 512),
             (1000, 20, 7), (61, 300, 1)], [1, 4, 22, 74], [1, 512, 768, 4096]):
        v = ao.Variant(G, fam, 64, R, bz, flags)
        got = ao.ao_jacobi_planes(v, nx, ny, nz, res)
        assert got == rule(nx, ny, nz, T, width, R, bz, res), (fam, nx, ny, nz, bz, res)
        assert 1 <= got <= min(bz, nz)


def test_known_picks():
    t4 = ao.Variant(G, ao.FAM_JACOBI_ZREG_T4, 64, 4, 74,
                    ao.AO_VF_NT_STORE | ao.AO_VF_STAGED | ao.AO_VF_FILL_Z)
    t3 = ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 64, 4, 22, ao.AO_VF_STAGED | ao.AO_VF_FILL_Z)
    # two four-sweep blocks per CU on 256 CUs: 512^3 keeps its 74 planes
    # (7 chunks, 4 rounds of 80 plane steps), 256^3 takes 43 (6 chunks of
    # 80 columns: 480 blocks, one round)
    assert ao.ao_jacobi_planes(t4, 512, 512, 512, 512) == 74
    assert ao.ao_jacobi_planes(t4, 256, 256, 256, 512) == 43
    # three three-sweep blocks per CU: 128^3 in chunks of 4
    assert ao.ao_jacobi_planes(t3, 128, 128, 128, 768) == 4
    # one resident block: as few chunks as the bound allows (5 for 300
    # planes), each as short as that count permits
    assert ao.ao_jacobi_planes(t4, 300, 300, 300, 1) == 60


def test_without_the_flag_the_declared_planes():
    for fam, T, width in FAMS:
        v = ao.Variant(G, fam, 64, 2, 13, ao.AO_VF_STAGED if T >= 3 else 0)
        assert ao.ao_jacobi_planes(v, 512, 512, 512, 512) == 13
        assert ao.ao_jacobi_planes(v, 5, 5, 5, 512) == 13


def test_refusals():
    ok = ao.Variant(G, ao.FAM_JACOBI_ZREG_T4, 64, 4, 74, ao.AO_VF_FILL_Z)
    bad = [ao.Variant(G, ao.FAM_JACOBI_DIRECT, 64, 4, 1, 0),          # not a z-march
           ao.Variant(G, ao.FAM_JACOBI_ZREG_T4, 64, 7, 74, 0),        # no kernel for 7 rows
           ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 128, 4, 22, 0),       # strips of 64 only
           ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 64, 4, 0, 0),         # no planes
           ao.Variant(G, ao.FAM_JACOBI_ZREG_T3, 64, 4, 22,
                      ao.AO_VF_STAGED | ao.AO_VF_HALO_PREFETCH),     # staged without prefetch
           ao.Variant(ao.AO_TARGET_HOST, ao.FAM_JACOBI_HOST, 64, 4, 1, 0)]
    for v in bad:
        with pytest.raises(ao.AdaptError):
            ao.ao_jacobi_planes(v, 64, 64, 64, 512)
    for dims in [(0, 4, 4), (4, -1, 4), (4, 4, 0)]:
        with pytest.raises(ao.AdaptError):
            ao.ao_jacobi_planes(ok, *dims, 512)


def test_declaration_refuses_the_flag_outside_the_z_marches():
    with pytest.raises(ao.AdaptError):
        ao.region_declare_variants("fill_on_direct", ao.AO_JACOBI7_F64,
                                   [ao.Variant(G, ao.FAM_JACOBI_DIRECT, 64, 4, 1, ao.AO_VF_FILL_Z)])
    h = ao.region_declare_variants("fill_on_t4", ao.AO_JACOBI7_F64,
                                   [ao.Variant(G, ao.FAM_JACOBI_ZREG_T4, 64, 4, 74,
                                               ao.AO_VF_STAGED | ao.AO_VF_FILL_Z)])
    ao.region_destroy(h)
