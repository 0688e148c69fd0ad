"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded float32 inputs.

Tolerances (the contract of the library):
  plain FP32 path:  relative energy error <= 1e-6, relative RMS force error <= 1e-5;
  BF16X3 path:      relative RMS force error <= 1e-3, relative energy error <= 1e-3
                    (the form's force budget; random charges reach ~1e-4 in energy).
The GPU evaluates the far part on a grid, so its error against the oracle's
exact image sums also contains the spreading discretisation (about 2e-6 in
force at the default 10^3 stencil with sigma_s = 0.9 h, under 1e-4 at the
BF16X3 default 6^3 with 0.74 h).
"""
import math

import numpy as np
import pytest

import oracle
from gpu_util import compare, gpu_eval, log, oracle_eval, oracle_params, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1911_01377_amd import (USERIES_BF16X3, USERIES_C0, USERIES_C1, USERIES_C2_B2,  # noqa: E402
                                  USERIES_TABLE1_ROW1, USERIES_TABLE1_ROW2, USERIES_TABLE1_ROW3,
                                  synth)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_random_cube_512_plain():
    xyz, q, box = synth.random_cube(512, 24.0, seed=1377)
    compare("random512/plain", xyz, q, box, 9.0, (32, 32, 32), 1e-6, 1e-5)


def test_random_cube_512_bf16x3():
    xyz, q, box = synth.random_cube(512, 24.0, seed=1377)
    compare("random512/bf16x3", xyz, q, box, 9.0, (32, 32, 32), 1e-3, 1e-3,
            precision=USERIES_BF16X3)


@pytest.mark.parametrize("n_mol", [300, 517])
def test_small_water_ragged_grid(n_mol):
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=50 + n_mol)
    g = int(np.ceil(L))
    compare("water%d/plain" % n_mol, xyz, q, box, min(9.0, 0.45 * L), (g, g, g), 1e-6, 1e-5)


def test_small_water_bf16x3():
    n_mol = 700
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=3)
    g = int(np.ceil(L))
    compare("water700/bf16x3", xyz, q, box, 9.0, (g, g, g), 1e-3, 1e-3,
            precision=USERIES_BF16X3)


@pytest.mark.parametrize("P,ratio", [(6, 0.9), (8, 0.9), (4, 0.83)])
def test_stencil_widths(P, ratio):
    """Non-default spreading stencils through the plain path: P = 6 and 8 take
    the gather kernel's 4^3 bricks (P > 5) and larger halos; every width sizes
    the gather kernel's LDS.  P >= 5 at sigma_s = 0.9 h meets the plain
    contract; the 8^3 stencil at 0.83 h (about 2e-5 in force on water) is held
    to 1e-4."""
    n_mol = 500
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=61)
    g = int(np.ceil(L))
    tol = (1e-6, 1e-5) if P >= 5 else (1e-4, 1e-4)
    compare("water500/plain/P%d" % P, xyz, q, box, min(9.0, 0.45 * L), (g, g, g), tol[0], tol[1],
            stencil_half=P, sigma_s_over_h=ratio)


def test_orthorhombic_box_and_grid():
    rng = np.random.default_rng(4)
    box = (20.0, 23.5, 27.0)
    n = 700
    xyz = (rng.uniform(0, 1, (n, 3)) * box).astype(np.float32)
    q = synth._quantise(rng.uniform(-1, 1, n))
    q[-1] = -np.sum(q[:-1])
    compare("ortho700/plain", xyz, q.astype(np.float32), box, 8.0, (20, 24, 30), 1e-6, 1e-5)


def test_tall_box_long_columns():
    # a 16 x 16 x 96 A water cell (six z-replicas of a 16 A water box): 9
    # columns of ~270 charges, so the column sort takes its bitonic path
    # (columns of up to 256 charges are ranked by counting)
    x1, q1, box1 = synth.water_box(n_mol=137, L=16.0, seed=29)
    L = box1[0]
    xyz = np.concatenate([x1 + np.array([0.0, 0.0, k * L], np.float32) for k in range(6)])
    q = np.concatenate([q1] * 6)
    box = (L, L, 6 * L)
    _, _, _, _, info = compare("tallwater/plain", xyz.astype(np.float32), q, box, 0.45 * L,
                               (16, 16, 96), 1e-6, 1e-5)
    assert len(q) / (info["ncell"][0] * info["ncell"][1]) > 256


def test_one_dense_column_global_ranking():
    """2,000 random charges in a 3 x 3 A wire along z of a 20 x 20 x 64 A cell:
    the 4 x 4 columns are 5 A wide, so one column holds every charge, more
    than the 1,024 that the column sort ranks in LDS (it ranks them from
    global memory), and the other fifteen are empty."""
    xyz, q, _ = synth.random_box(2000, (3.0, 3.0, 64.0), seed=43)
    xyz = (xyz + np.array([0.5, 0.5, 0.0], np.float32)).astype(np.float32)
    box = (20.0, 20.0, 64.0)
    _, _, _, _, info = compare("wire2000/plain", xyz, q, box, 9.0, (20, 20, 64), 1e-6, 1e-5,
                               e_scale="parts")
    assert tuple(info["ncell"][:2]) == (4, 4), info["ncell"]


def test_many_columns_global_binning():
    """A flat 256 x 256 x 19 A cell of 200,000 random charges: 69 x 69
    columns, more than the 4096 whose counts the binning kernels keep in LDS,
    so the column counts, the slot counters and the offsets (scan kernel) take
    their global-memory paths.  The oracle's full O(n^2) sum is out of reach
    at this size: forces on 128 sampled charges are compared (each an O(n)
    oracle sum), and the force sum must vanish up to rounding.  The x-y grid
    spacing is 2 A (0.95 A in z)."""
    xyz, q, box = synth.random_box(200000, (256.0, 256.0, 19.0), seed=31)
    rc, grid = 9.0, (128, 128, 20)
    log("case manycols/plain: n=%d box=%s rc=%g grid=%s" % (len(q), box, rc, grid))
    _, gf, info = gpu_eval(xyz, q, box, rc, grid)
    ncol = info["ncell"][0] * info["ncell"][1]
    assert ncol > 4096, info["ncell"]
    idx = np.random.default_rng(3).choice(len(q), 128, replace=False)
    fo = oracle.forces_subset(xyz.astype(np.float64), q.astype(np.float64), box,
                              oracle_params(info, rc), idx)
    df = rel_rms(gf[idx], fo)
    rms = float(np.sqrt(np.mean(np.sum(gf ** 2, axis=1))))
    mag = np.sqrt(np.sum(fo ** 2, axis=1))
    da = float((np.sqrt(np.sum((gf[idx] - fo) ** 2, axis=1)) / np.maximum(mag, rms)).max())
    fsum = float(np.linalg.norm(gf.sum(axis=0)))
    log("   columns %s, dF(128 sampled)=%.2e, max|dF_i|/max(|F_i|,rms)=%.2e, |sum F|=%.3e (rms %.3e)"
        % (info["ncell"], df, da, fsum, rms))
    assert df <= 1e-5
    assert da <= 1e-4
    assert fsum <= 1e-3 * math.sqrt(len(q)) * rms


FORMS = [(0, (1e-6, 1e-5)), (USERIES_BF16X3, (1e-3, 1e-3))]


def _form(precision):
    return "bf16x3" if precision else "plain"


@pytest.mark.parametrize("precision,tol", FORMS)
def test_many_candidates_per_cluster(precision, tol):
    """3,000 random charges in a 20 A cube (0.375 per A^3) with r_c = 9.5 A:
    every cluster has 2,400 to 3,000 candidates (a host count with the
    kernel's column and z-window rules), more than the 2,048 whose ranges
    the pair kernel looks up in its table, so every block takes the range
    search instead."""
    xyz, q, box = synth.random_box(3000, (20.0, 20.0, 20.0), seed=47)
    compare("dense3000/" + _form(precision), xyz, q, box, 9.5, (20, 20, 20), tol[0], tol[1],
            e_scale="parts", precision=precision)


@pytest.mark.parametrize("precision,tol", FORMS)
def test_terms_staged_in_chunks(precision, tol):
    """N = 4 on grids of 128 z points: a z-convolution block stages the columns
    of at most 2 terms at once (20 KiB of LDS), so it runs over two chunks of
    terms, in both forms.  A 32 A water box (32 x 32 x 128 grid) is held to
    the form's tolerances.  The second chunk's terms (16 and 32 A wide) must
    be in the result: for 2000 random charges in a 32 A cube, whose far energy
    they move by about 1%, the far energy lies within a fifth of the gap
    between the oracle's 4-term value and its value from the first 2 terms."""
    xyz, q, box = synth.water_box(None, 32.0, seed=23)
    _, _, _, _, info = compare("chunks/%s" % _form(precision), xyz, q, box, 8.0, (32, 32, 128),
                               tol[0], tol[1], n_terms=4, precision=precision)
    assert info["n_terms"] == 4 and info["n_terms_grid"] == 4
    xyz, q, box = synth.random_cube(2000, 32.0, seed=5)
    gp, _, info = gpu_eval(xyz, q, box, 8.0, (48, 48, 128), n_terms=4, precision=precision)
    x64, q64 = xyz.astype(np.float64), q.astype(np.float64)
    far4, _ = oracle.eval_far(x64, q64, box, oracle_params(info, 8.0))
    far2, _ = oracle.eval_far(x64, q64, box, oracle_params(dict(info, n_terms=2), 8.0))
    log("   random2000 far energy: gpu %.9f, oracle 4 terms %.9f, first 2 only %.9f"
        % (gp[1], far4, far2))
    assert abs(gp[1] - far4) < 0.2 * abs(far4 - far2)


@pytest.mark.parametrize("precision,tol", FORMS)
def test_terms_wider_than_the_box_are_skipped(precision, tol):
    """N = 8 in a 30 A water box: terms 4..7 (64 to 515 A wide) have every
    non-zero Fourier mode below 2^-60 of their k = 0 mode, so the grid
    evaluates terms 0..3 only; the oracle sums all eight.  Evaluated on the
    grid, those terms' nearly constant values would only add FP32 rounding
    (about 5e-6 of the far energy at N = 8)."""
    xyz, q, box = synth.water_box(None, 30.0, seed=24)
    _, _, _, _, info = compare("wide/%s" % _form(precision), xyz, q, box, 8.0, (32, 32, 32),
                               tol[0], tol[1], n_terms=8, precision=precision)
    assert info["n_terms"] == 8 and info["n_terms_grid"] == 4


@pytest.mark.parametrize("k", range(6))
@pytest.mark.parametrize("precision,tol", FORMS)
def test_random_water_configurations(k, precision, tol):
    """Seeded random water boxes: 200-1,200 molecules (L = 18-33 A), a grid
    spacing drawn per axis from [0.75, 0.95] A (grids of any length, not
    multiples of the tile sizes), r_c = min(9, 0.45 L), the default series."""
    rng = np.random.default_rng(1000 + k)
    n_mol = int(rng.integers(200, 1201))
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=2000 + k)
    grid = tuple(int(np.ceil(L / rng.uniform(0.75, 0.95))) for _ in range(3))
    compare("randwater%d/%s" % (k, _form(precision)), xyz, q, box, min(9.0, 0.45 * L), grid,
            tol[0], tol[1], precision=precision)


@pytest.mark.parametrize("precision,tol", FORMS)
def test_non_neutral_and_single_charge(precision, tol):
    """A net charge Q: the far part sums only k != 0 (eqs. 4, 9, 10), so any
    uniform offset of the grid potential (left by the spreading weights' sums
    and the FP32 rounding of the widest terms) must not reach the energy, where
    it would enter as Q x offset / 2.  Held to the form's neutral-input
    tolerances, together with a single charge (the simple-cubic Wigner
    lattice)."""
    rng = np.random.default_rng(8)
    L = 18.0
    xyz = rng.uniform(0, L, (200, 3)).astype(np.float32)
    q = (rng.uniform(-1, 1, 200) + 0.05).astype(np.float32)
    f = _form(precision)
    compare("nonneutral200/" + f, xyz, q, (L, L, L), 8.0, (24, 24, 24), tol[0], tol[1],
            precision=precision)
    q2 = (rng.uniform(-1, 1, 300) + 0.3).astype(np.float32)
    xyz2 = rng.uniform(0, 22.0, (300, 3)).astype(np.float32)
    compare("nonneutral300/" + f, xyz2, q2, (22.0, 22.0, 22.0), 9.0, (22, 22, 22), tol[0], tol[1],
            precision=precision)
    compare("single/" + f, np.array([[1.0, 2.0, 3.0]], np.float32), np.array([1.0], np.float32),
            (L, L, L), 8.0, (24, 24, 24), tol[0], tol[1], precision=precision)


def test_empty_input():
    log("case empty")
    parts, f, _ = gpu_eval(np.zeros((0, 3), np.float32), np.zeros(0, np.float32),
                           (20.0, 20.0, 20.0), 8.0, (20, 20, 20))
    assert np.all(parts == 0.0) and f.shape == (0, 3)


def test_images_and_permutation():
    xyz, q, box = synth.random_cube(300, 21.0, seed=12)
    # positions on a 2^-12 A lattice, so that adding whole box lengths is exact in float32
    xyz = (np.round(xyz.astype(np.float64) * 4096) / 4096).astype(np.float32)
    log("case images/permutation")
    p0, f0, _ = gpu_eval(xyz, q, box, 9.0, (24, 24, 24))
    shift = np.array([21.0, -42.0, 63.0], np.float32)
    p1, f1, _ = gpu_eval(xyz + shift, q, box, 9.0, (24, 24, 24))
    assert abs(p1[4] - p0[4]) <= 1e-9 * abs(p0[4])
    assert np.max(np.abs(f1 - f0)) <= 1e-6 * np.max(np.abs(f0))
    perm = np.random.default_rng(1).permutation(len(q))
    p2, f2, _ = gpu_eval(xyz[perm], q[perm], box, 9.0, (24, 24, 24))
    assert abs(p2[4] - p0[4]) <= 1e-7 * abs(p0[4])
    assert rel_rms(f2, f0[perm]) <= 1e-6


def test_repeat_is_bitwise_identical():
    import torch as T
    from paper_1911_01377_amd import Plan
    log("case determinism")
    xyz, q, box = synth.water_box(n_mol=800, L=(800 / synth.WATER_DENSITY) ** (1 / 3), seed=9)
    plan = Plan(box, 9.0, (29, 29, 29))
    x = T.from_numpy(xyz).cuda()
    qq = T.from_numpy(q).cuda()
    e1, f1, _ = plan.eval(x, qq)
    e1, f1 = e1.clone(), f1.clone()
    for _ in range(3):
        e2, f2, _ = plan.eval(x, qq)
    T.cuda.synchronize()
    assert T.equal(e1, e2) and T.equal(f1, f2)
    plan.close()


def test_near_and_far_parts_separately():
    """The near energy matches the oracle's pair sum; the far energy its image sums."""
    xyz, q, box = synth.random_cube(400, 22.0, seed=31)
    log("case parts")
    gp, gf, info = gpu_eval(xyz, q, box, 9.0, (30, 30, 30))
    op, of = oracle_eval(xyz, q, box, info, 9.0)
    # the total of random charges is a small difference of much larger parts,
    # so the parts are measured against the sum of their magnitudes
    scale = abs(op["near"]) + abs(op["far"]) + abs(op["total"])
    log("   near %.3e far %.3e (x scale)" % (abs(gp[0] - op["near"]) / scale,
                                            abs(gp[1] - op["far"]) / scale))
    assert abs(gp[0] - op["near"]) <= 1e-6 * scale
    assert abs(gp[1] - op["far"]) <= 1e-6 * scale
    assert abs(gp[2] - op["self"]) <= 1e-12 * op["self"]


def test_graph_replay_matches_eager():
    """One evaluation captured in a HIP graph (as the benchmark times it):
    every replay, with eager evaluations between them, gives the eager result
    bitwise."""
    from paper_1911_01377_amd import Plan
    xyz, q, box = synth.water_box(n_mol=400, L=(400 / synth.WATER_DENSITY) ** (1 / 3), seed=71)
    g = int(np.ceil(box[0]))
    log("case graph replay: n=%d grid=%d" % (len(q), g))
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    qq = torch.from_numpy(q).to(dev)
    for prec in (0, USERIES_BF16X3):
        plan = Plan(box, min(9.0, 0.45 * box[0]), (g, g, g), precision=prec)
        e_ref, f_ref, _ = plan.eval(x, qq)
        torch.cuda.synchronize()
        e_ref, f_ref = e_ref.clone(), f_ref.clone()
        forces = torch.empty_like(f_ref)
        energy = torch.empty_like(e_ref)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.eval(x, qq, forces, energy)
        for rep in range(4):
            forces.zero_()
            energy.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(forces, f_ref) and torch.equal(energy, e_ref), (prec, rep)
            e2, f2, _ = plan.eval(x, qq)       # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(f2, f_ref) and torch.equal(e2, e_ref)
        plan.close()


CONSTRUCTIONS = [(USERIES_C0, "C0"), (USERIES_C2_B2, "C2b2"), (USERIES_TABLE1_ROW1, "T1r1"),
                 (USERIES_TABLE1_ROW2, "T1r2"), (USERIES_TABLE1_ROW3, "T1r3")]


@pytest.mark.parametrize("construction,name", CONSTRUCTIONS)
@pytest.mark.parametrize("precision,tol", FORMS)
def test_every_construction(construction, name, precision, tol):
    """Every construction the plan accepts, through the same kernels, at the
    form's tolerances: C0 (eqs. 19-21), the C2 series of eq. 28 with Table 2's
    b = 2 parameters, and the three C2 points of the C1 construction in
    Table 1 (b = 1.63, 1.32, 1.22: sigma = r_c / r0 down to 1.6 A, N up to
    15 terms, and the narrowest Gaussians evaluated exactly in the near part).
    A water box and a box of random charges each; the oracle takes the plan's
    (b, sigma, w0, s0, N).

    The grid spacing follows the narrowest far Gaussian s_0 = sigma s0: at most
    1 A and at most s_0 / 2.  Spreading, convolution and gathering represent
    s_0 through Gaussians narrower still (sigma_s and the on-grid kernel), so
    a grid much coarser than s_0 / 2 loses the far part's accuracy (Table 1
    row 3 at r_c = 9 A has s_0 = 1.6 A: the FP64 discrete scheme misses the
    exact far energy by 8e-6 of the total at h = 0.61 s_0 and by 4e-8 at
    0.50 s_0)."""
    from paper_1911_01377_amd import _native
    _, r0, _, s0 = _native.useries_solve_construction(construction, 2.0)
    s_min = 9.0 / r0 * s0
    n_mol = 600
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=300 + construction)
    g = int(np.ceil(L / min(1.0, 0.5 * s_min)))
    f = _form(precision)
    _, _, _, _, info = compare("water600/%s/%s" % (name, f), xyz, q, box, 9.0, (g, g, g),
                               tol[0], tol[1], construction=construction, precision=precision)
    if construction in (USERIES_TABLE1_ROW2, USERIES_TABLE1_ROW3) and not precision:
        assert info["near_exact"] > 0
    # random charges: the total energy is a small difference of the parts
    # (random512 with Table 1 row 2: near 3.9, far 30.8, self 36.3, total
    # -1.6), so the energy is held relative to the parts' magnitudes; with N = 10
    # terms the FP32 far part errs by about 2.5e-7 of itself, and the BF16X3
    # form's 6^3 stencil truncates its Gaussians at 4 sigma_s (2.7e-4 of the
    # far part)
    xyz, q, box = synth.random_cube(512, 24.0, seed=400 + construction)
    g = max(32, int(np.ceil(24.0 / (0.5 * s_min))))
    compare("random512/%s/%s" % (name, f), xyz, q, box, 9.0, (g, g, g), tol[0], tol[1],
            e_scale="parts", construction=construction, precision=precision)


def test_c1_at_other_bases():
    """The C1 construction solved on the host for b other than 2 (the
    smallest root of eq. 26 with w0 from eq. 25): b = 1.5 and 3."""
    n_mol = 500
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=77)
    g = int(np.ceil(L))
    for b in (1.5, 3.0):
        compare("water500/C1/b%.1f" % b, xyz, q, box, min(9.0, 0.45 * L), (g, g, g), 1e-6, 1e-5,
                construction=USERIES_C1, b=b)


@pytest.mark.parametrize("precision,tol", FORMS)
def test_dispersion_kernel_alpha6(precision, tol):
    """The 1/r^6 series (App. A, C1 construction for 1/r^6 at b = 2) through
    the same kernels: positive coefficients (no neutrality; the far terms keep
    their k = 0 components), a water box with one coefficient per site kind
    and random coefficients in a cube; against the oracle's 1/r^6 series with
    the plan's parameters."""
    f = _form(precision)
    n_mol = 600
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, _, box = synth.water_box(n_mol=n_mol, L=L, seed=66)
    c = np.tile(np.array([1.0, 0.25, 0.25], np.float32), n_mol)
    g = int(np.ceil(L))
    _, _, _, _, info = compare("water600/r^-6/" + f, xyz, c, box, 9.0, (g, g, g), tol[0], tol[1],
                               alpha=6, precision=precision)
    assert info["n_terms"] >= 2
    rng = np.random.default_rng(67)
    xyz = rng.uniform(0, 22.0, (700, 3)).astype(np.float32)
    c = rng.uniform(0.2, 1.5, 700).astype(np.float32)
    compare("random700/r^-6/" + f, xyz, c, (22.0, 22.0, 22.0), 8.5, (24, 24, 24), tol[0], tol[1],
            alpha=6, precision=precision)


@pytest.mark.parametrize("precision,tol", FORMS)
def test_repulsion_kernel_alpha12(precision, tol):
    """The 1/r^12 series (App. A, C1 construction for 1/r^12 at b = 2,
    mellin factor 3840) through the same kernels: a water box with one
    coefficient per site kind (close intramolecular pairs dominate) and random
    positive coefficients in a cube; against the oracle's 1/r^12 series with
    the plan's parameters."""
    f = _form(precision)
    n_mol = 600
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, _, box = synth.water_box(n_mol=n_mol, L=L, seed=68)
    c = np.tile(np.array([1.0, 0.1, 0.1], np.float32), n_mol)
    g = int(np.ceil(L))
    _, _, _, _, info = compare("water600/r^-12/" + f, xyz, c, box, 9.0, (g, g, g), tol[0], tol[1],
                               alpha=12, precision=precision)
    assert info["n_terms"] >= 1
    rng = np.random.default_rng(69)
    xyz = rng.uniform(0, 22.0, (700, 3)).astype(np.float32)
    c = rng.uniform(0.2, 1.5, 700).astype(np.float32)
    compare("random700/r^-12/" + f, xyz, c, (22.0, 22.0, 22.0), 8.5, (24, 24, 24), tol[0], tol[1],
            alpha=12, precision=precision)


@pytest.mark.parametrize("alpha", [6, 12])
def test_power_kernels_in_a_non_cubic_cell(alpha):
    """1/r^6 and 1/r^12 (App. A) in a 22 x 24 x 26 A cell: the three axes
    have different fixed-point scales, so the pair kernel scales each
    distance component to A with its own hi/lo scale pair (the cubic path
    keeps them in units); random positive coefficients, both forms, against
    the oracle."""
    rng = np.random.default_rng(70 + alpha)
    box = (22.0, 24.0, 26.0)
    xyz = (rng.uniform(0, 1, (900, 3)) * np.array(box)).astype(np.float32)
    c = rng.uniform(0.2, 1.5, 900).astype(np.float32)
    for precision, tol in FORMS:
        compare("noncubic900/r^-%d/%s" % (alpha, _form(precision)), xyz, c, box, 9.0, (24, 24, 27),
                tol[0], tol[1], alpha=alpha, precision=precision)


def test_repulsion_lattice_forces_vanish():
    """Identical coefficients on a simple-cubic lattice (64 sites, spacing
    2 A): the 1/r^12 forces vanish by symmetry and the energy matches the
    oracle's."""
    g = np.arange(8) * 2.0
    xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    c = np.ones(len(xyz), np.float32)
    box = (16.0, 16.0, 16.0)
    log("case sc512/r^-12")
    gp, gf, info = gpu_eval(xyz, c, box, 7.9, (16, 16, 16), alpha=12)
    op, of = oracle_eval(xyz, c, box, info, 7.9, alpha=12)
    de = abs(gp[4] - op["total"]) / abs(op["total"])
    fpair = 12.0 / 2.0 ** 13
    log("   E_gpu=%.12g E_oracle=%.12g dE=%.2e max|F_gpu|=%.2e max|F_oracle|=%.2e (pair %.2e)"
        % (gp[4], op["total"], de, np.max(np.abs(gf)), np.max(np.abs(of)), fpair))
    assert de <= 1e-6
    assert np.max(np.abs(of)) < 1e-12 * fpair
    assert np.max(np.abs(gf)) < 1e-5 * fpair


def test_dispersion_lattice_forces_vanish():
    """Identical coefficients on a simple-cubic lattice (64 sites, spacing
    4 A): the 1/r^6 forces vanish by symmetry and the energy matches the
    oracle's."""
    g = np.arange(4) * 4.0
    xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    c = np.ones(len(xyz), np.float32)
    box = (16.0, 16.0, 16.0)
    log("case sc64/r^-6")
    gp, gf, info = gpu_eval(xyz, c, box, 7.9, (16, 16, 16), alpha=6)
    op, of = oracle_eval(xyz, c, box, info, 7.9, alpha=6)
    de = abs(gp[4] - op["total"]) / abs(op["total"])
    # a typical pair force at the lattice spacing, for scale
    fpair = 6.0 / 4.0 ** 7
    log("   E_gpu=%.12g E_oracle=%.12g dE=%.2e max|F_gpu|=%.2e max|F_oracle|=%.2e (pair %.2e)"
        % (gp[4], op["total"], de, np.max(np.abs(gf)), np.max(np.abs(of)), fpair))
    assert de <= 1e-6
    assert np.max(np.abs(of)) < 1e-12 * fpair
    assert np.max(np.abs(gf)) < 1e-5 * fpair


@pytest.mark.parametrize("precision,tol", FORMS)
def test_spectral_wide_terms(precision, tol):
    """The widest far terms applied together in spectral form (a low-rank form
    of their circulants: the real Fourier modes each needs down to 1e-9 of its
    first mode), against the oracle's exact image sums: a 30 A water box at
    b = 2 (N = 3, the two widest spectral), the same with N = 8 terms, and
    Table 1 row 3 (N = 15, the eight widest spectral).  The spectral and
    dense forms of one plan agree to the truncation (1e-9) plus FP32
    rounding."""
    f = _form(precision)
    xyz, q, box = synth.water_box(None, 30.0, seed=24)
    for nt in (0, 8):
        _, gf, _, of, info = compare("wide30/spectral/N%d/%s" % (nt, f), xyz, q, box, 9.0,
                                     (30, 30, 30), tol[0], tol[1], n_terms=nt, spectral=1,
                                     precision=precision)
        assert info["n_terms_spectral"] >= 2, info
        assert info["n_terms_grid"] - info["n_terms_spectral"] >= 1
        gd, fd, infod = gpu_eval(xyz, q, box, 9.0, (30, 30, 30), n_terms=nt, spectral=0,
                                 precision=precision)
        log("   spectral %d of %d grid terms, ranks %s; vs the dense form: dF=%.2e"
            % (info["n_terms_spectral"], info["n_terms_grid"], info["spectral_rank"],
               rel_rms(gf, fd)))
        assert rel_rms(gf, fd) < (2e-6 if not precision else 1e-4)
    n_mol = 600
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=313)
    _, _, _, _, info = compare("water600/T1r3/spectral/" + f, xyz, q, box, 9.0, (33, 33, 33),
                               tol[0], tol[1], construction=USERIES_TABLE1_ROW3, spectral=1,
                               precision=precision)
    assert info["n_terms_spectral"] >= 2, info
