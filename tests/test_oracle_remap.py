"""Independent pins of the oracle's response-row decisions.

The oracle's response row of a sub-segment (2D) or sub-patch (3D) decides,
for every neighbouring crystal, which table entry it reads: the angle row
(nearest row of the incidence angle), the sub-position, the mirror for
photons leaning towards lower crystal indices, and -- for crystals of the
next block -- the two-block remap of Sec 2.1.2 (Eq.2, 4, 5): the virtual
crystal the ray enters behind the next block's face line, its entry
sub-position, the table offset of each real crystal, the angle row of the
next block's incidence angle, and in 3D the axial carry (ring and axial
sub-position where the ray meets the next block's face).

Here each of those decisions is re-derived by tracing the ray with plain
vector geometry, in a frame where the photon leans towards increasing
coordinates: the ray from the voxel centre through the sub-segment centre is
intersected with the next block's face line, the crystal lattice of that
block is extended past its near edge, and the cell holding the intersection
gives the virtual crystal and the entry sub-position.  No formula of Eq.4 or
Eq.5 is used.  The oracle is called with a marker table whose every entry is
its own index plus one, so the response row's values name the entries read;
both they and the returned indices must equal the traced ones, entry by
entry, except for decisions the oracle flags as within a hair of a boundary.
"""
import math

import numpy as np
import pytest

from paper_1607_06170_amd import synth as S

NARROW = S.CFG_2D_NARROW
WIDE = S.CFG_2D
# the small 3D scanner's transaxial ring as a 2D ring (12 blocks of 4 x 2 mm, faces at 16 mm)
SMALL_RING = dict(S.CFG_3D_SMALL, n_cz=1, n_brings=1, nz=1)


def _frame(cfg, b):
    phi = cfg["phi0"] + 2.0 * math.pi * (b % cfg["n_blocks"]) / cfg["n_blocks"]
    return np.array([math.cos(phi), math.sin(phi)]), np.array([-math.sin(phi), math.cos(phi)])


def _cell(eta, width, n_cells):
    """Cell of a lattice of `width` whose cell 0 starts at -n_cells*width/2:
    (index, offset from the cell's lower edge); indices past either end are
    the lattice extended beyond the block."""
    q = (eta + 0.5 * n_cells * width) / width
    k = math.floor(q)
    return k, (q - k) * width


def _round_row(angle_rad, step_deg):
    return math.floor(abs(angle_rad) * 180.0 / math.pi / step_deg + 0.5)


def traced_row_2d(cfg, P, step, v, g, p):
    """Table entry index (row * P + p) * 5 + offset + 2 read for each crystal
    g + a (a = -2..2), or -1, from a ray trace."""
    nc, lam, rf, R = cfg["n_ct"], cfg["pitch_t"], cfg["r_face"], cfg["n_blocks"]
    W = nc * lam
    b, c = divmod(g, nc)
    n0, t0 = _frame(cfg, b)
    xi_m = -0.5 * W + (c + (p + 0.5) / P) * lam
    m = rf * n0 + xi_m * t0
    d = m - np.asarray(v, dtype=np.float64)
    d /= np.linalg.norm(d)
    alpha = math.atan2(d @ t0, d @ n0)
    sg = 1 if alpha >= 0 else -1          # local frame: the photon leans towards +eta
    cl, u = _cell(sg * xi_m, lam, nc)     # entry crystal and sub-position in the local frame
    pl = math.floor(u * P / lam)
    row = _round_row(alpha, step)
    out = []
    for a in range(-2, 3):
        al = sg * a
        ccl = cl + al
        if 0 <= ccl < nc:
            out.append((row * P + pl) * 5 + al + 2)
            continue
        if ccl < 0:                       # behind the receding edge: across a gap, no response
            out.append(-1)
            continue
        n1, t1 = _frame(cfg, b + sg)      # the block the photon leans towards
        beta = math.atan2(sg * (d @ t1), d @ n1)
        if not beta > 0.0:                # the ray turns away from the next block's crystals
            out.append(-1)
            continue
        s = (rf - np.asarray(v) @ n1) / (d @ n1)
        p1 = np.asarray(v) + s * d        # where the ray meets the next block's face line
        mv, u1 = _cell(sg * (p1 @ t1), lam, nc)
        assert mv < 0, "the ray meets the next face line before that block's crystals"
        idx = (ccl - nc) - mv             # lattice cells from the virtual entry crystal to the real one
        if idx > 2:
            out.append(-1)
            continue
        out.append((_round_row(beta, step) * P + math.floor(u1 * P / lam)) * 5 + idx + 2)
    return out


def _marker_table(oracle, n):
    return np.arange(n, dtype=np.float64) + 1.0


@pytest.mark.parametrize("cfg,n_rows", [(NARROW, 61), (WIDE, 61), (SMALL_RING, 91)])
def test_response_rows_2d_match_ray_trace(oracle, cfg, n_rows):
    P, step = 4, 1.0
    tab = oracle.TableRef(_marker_table(oracle, n_rows * P * 5).reshape(n_rows, P, 5), n_rows, P, step)
    nx, ny = cfg["nx"], cfg["ny"]
    rng = np.random.default_rng(11)
    vox = rng.choice(nx * ny, 24, replace=False)
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    n_cmp = n_remap = n_mirror_remap = 0
    for vid in vox:
        v = oracle.voxel_centre(cfg, int(vid))[:2]
        for g in range(Nc):
            for p in range(P):
                val, src, fl = oracle.uv_row_2d(cfg, tab, v, g, p)
                if fl & (oracle.F_TIES | oracle.F_RANGE):
                    continue
                exp = traced_row_2d(cfg, P, step, v, g, p)
                assert list(src) == exp, (vid, g, p, list(src), exp)
                assert np.array_equal(val, np.where(src >= 0, src + 1.0, 0.0))
                n_cmp += 1
                # entries read for crystals of the neighbouring block
                c = g % cfg["n_ct"]
                for a in range(-2, 3):
                    if exp[a + 2] >= 0 and not 0 <= c + a < cfg["n_ct"]:
                        n_remap += 1
                        n_mirror_remap += a < 0
    assert n_cmp > 1000
    if cfg is not WIDE:   # the narrow gaps send photons into the next block, on both edges
        assert n_remap > 50 and n_mirror_remap > 20, (n_remap, n_mirror_remap)


def traced_row_3d(cfg, P, nr, step, c, g, pt, r, pz):
    """Table entry index of the 3D table read for each crystal (g + a_t, r + a_z),
    as a 5 x 5 array (-1: none), from a ray trace."""
    nc, lt, lz, rf = cfg["n_ct"], cfg["pitch_t"], cfg["pitch_z"], cfg["r_face"]
    NR = cfg["n_cz"] * cfg["n_brings"]
    W = nc * lt
    c = np.asarray(c, dtype=np.float64)
    b, cr = divmod(g, nc)
    n0, t0 = _frame(cfg, b)
    xi_m = -0.5 * W + (cr + (pt + 0.5) / P) * lt
    z_m = (r + (pz + 0.5) / P) * lz - 0.5 * NR * lz
    m = np.array([*(rf * n0 + xi_m * t0), z_m])
    d = m - c
    dh = d[:2]
    at_, az_ = math.atan2(dh @ t0, dh @ n0), math.atan2(d[2], dh @ n0)
    st, sz = (1 if at_ >= 0 else -1), (1 if az_ >= 0 else -1)
    ctl, ut = _cell(st * xi_m, lt, nc)
    rl, uz = _cell(sz * z_m, lz, NR)
    ptl, pzl = math.floor(ut * P / lt), math.floor(uz * P / lz)

    def idx3(rt, rz, p_t, p_z, a_t, a_z):
        return ((((rt * nr + rz) * P + p_t) * P + p_z) * 5 + a_t + 2) * 5 + a_z + 2

    out = -np.ones((5, 5), dtype=np.int64)
    remap = None
    for a_t in range(-2, 3):
        for a_z in range(-2, 3):
            if not 0 <= r + a_z < NR:
                continue
            atl, azl = st * a_t, sz * a_z
            ccl = ctl + atl
            if 0 <= ccl < nc:
                out[a_t + 2, a_z + 2] = idx3(_round_row(at_, step), _round_row(az_, step), ptl, pzl, atl, azl)
                continue
            if ccl < 0:
                continue
            if remap is None:   # trace once into the next block
                n1, t1 = _frame(cfg, b + st)
                bt = math.atan2(st * (dh @ t1), dh @ n1)
                if not bt > 0.0:
                    remap = False
                else:
                    s = (rf - c[:2] @ n1) / (dh @ n1)
                    p1 = c + s * d
                    mv, u1 = _cell(st * (p1[:2] @ t1), lt, nc)
                    rl1, u1z = _cell(sz * p1[2], lz, NR)
                    bz = math.atan2(abs(d[2]), dh @ n1)   # axial angle in the next block's frame
                    remap = (mv, rl1 - rl, _round_row(bt, step), _round_row(bz, step), math.floor(u1 * P / lt),
                             math.floor(u1z * P / lz))
            if remap is False:
                continue
            mv, dr, rbt, rbz, p1t, p1z = remap
            idx, az1 = (ccl - nc) - mv, azl - dr
            if idx <= 2 and -2 <= az1 <= 2:
                out[a_t + 2, a_z + 2] = idx3(rbt, rbz, p1t, p1z, idx, az1)
    return out, remap


@pytest.mark.parametrize("which", ["small", "full"])
def test_response_rows_3d_match_ray_trace(oracle, which):
    P, step = 4, 1.0
    if which == "small":
        cfg, nr = S.CFG_3D_SMALL, 91
    else:
        cfg, nr = S.CFG_3D, 61
    tab = oracle.TableRef(_marker_table(oracle, nr * nr * P * P * 25).reshape(nr, nr, P, P, 5, 5), nr, P, step)
    NR = cfg["n_cz"] * cfg["n_brings"]
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    rng = np.random.default_rng(12)
    nvox = cfg["nx"] * cfg["ny"] * cfg["nz"]
    vox = rng.choice(nvox, 8, replace=False)
    n_cmp = n_remap = n_carry = 0
    for vid in vox:
        c = oracle.voxel_centre(cfg, int(vid))
        # sub-patches at block edges (where the remap acts) and a random spread elsewhere
        nc = cfg["n_ct"]
        keys = []
        for _ in range(3000):
            b = int(rng.integers(cfg["n_blocks"]))
            cr = int(rng.choice([0, 1, nc - 2, nc - 1])) if rng.random() < 0.8 else int(rng.integers(nc))
            if rng.random() < 0.5:   # steep axial rays near a ring's far edge: the axial carry
                r = int(rng.choice([0, 1, NR - 2, NR - 1]))
                pz = P - 1 if r >= NR // 2 else 0
            else:
                r, pz = int(rng.integers(NR)), int(rng.integers(P))
            keys.append((b * nc + cr, int(rng.integers(P)), r, pz))
        for (g, pt, r, pz) in keys:
            val, src, fl = oracle.uv_row_3d(cfg, tab, c, g, pt, r, pz)
            if fl & (oracle.F_TIES | oracle.F_RANGE):
                continue
            exp, remap = traced_row_3d(cfg, P, nr, step, c, g, pt, r, pz)
            assert np.array_equal(src, exp), (vid, g, pt, r, pz, src, exp)
            assert np.array_equal(val, np.where(src >= 0, src + 1.0, 0.0))
            n_cmp += 1
            cr = g % cfg["n_ct"]
            used = sum(int(exp[at + 2, az + 2] >= 0) for at in range(-2, 3) for az in range(-2, 3)
                       if not 0 <= cr + at < cfg["n_ct"])
            n_remap += used
            n_carry += used > 0 and remap[1] != 0   # the ray enters the next block in another ring
    assert n_cmp > 2000
    assert n_remap > 100, n_remap
    assert n_carry > 10, n_carry
