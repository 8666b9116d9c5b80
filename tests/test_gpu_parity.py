"""GPU (HIP, gfx950) path against the CPU oracle, element by element.

Tolerances (relative, max-norm over the field: max|X - X_ref| / max|X_ref|;
wall forces: 2-norm per group and variant): FP64 storage 1e-12; FP32 storage
1e-5 on fields and 1e-4 on wall forces; 16-bit storage 2e-3.

16-bit storage is compared with the oracle's FP64 arithmetic carrying the
same documented storage rounding (d*2^10/w in FP16, d/w in BF16, applied
wherever the library stores a state).  Its accuracy against the unquantized
FP64 oracle is stated separately (test_16bit_accuracy_vs_fp64).  Results
that miss their target are recorded as not met (MISS_QUANT, MISS_VS_FP64):
the test then ends as an expected failure stating the measured values, each
held to a recorded bound.
"""
import sys

import numpy as np
import pytest

from closed_forms import channel_recurrence
from helpers import check_targets, make_oracle, quantize_state, quantized_steps, rel_inf
from paper_2512_12213_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FIELD = {W.F64: 1e-12, W.F32: 1e-5, W.F16: 2e-3, W.BF16: 2e-3}
TOL_STRESS = {W.F64: 1e-12, W.F32: 1e-5, W.F16: 2e-3, W.BF16: 2e-3}
TOL_WALL = {W.F64: 1e-12, W.F32: 1e-4, W.F16: 2e-3, W.BF16: 2e-3}

# Recorded as not met: BF16 keeps 8 significant bits, so its rounding unit
# 2^-8 = 3.9e-3 exceeds the 2e-3 target and a single rounding that lands on
# the other side of a tie than in the quantized oracle already misses it; the
# stress, a small difference of stored values, carries that unit times
# |d| / |Pi^neq|.  Bounds (regression checks): two rounding units on fields
# and wall forces, 2e-2 on the stress.
MISS_QUANT = {W.F64: {}, W.F32: {}, W.F16: {},
              W.BF16: {"rho": 8e-3, "v": 8e-3, "sigma": 2e-2, "S": 2e-2, "wall": 8e-3, "state": 8e-3}}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_12213_amd import lbm as L
    L.lib()
    return L


def gpu_from(w, lbm, storage=None, u0=None, init=True):
    return lbm.from_workload(w, storage=storage, u0=u0, init=init)


def compare_all(g, o, storage, groups, what=""):
    rg, vg = g.get_macro()
    ro, vo = o.get_macro()
    tf = TOL_FIELD[storage]
    e_rho = np.abs(rg - ro).max()
    e_v = rel_inf(vg, vo)
    sg, Sg = g.stress()
    so, So = o.stress()
    e_s = rel_inf(sg, so)
    e_S = rel_inf(Sg, So)
    fg = g.wall_force()[:groups]
    fo = o.wall_force(groups)
    e_f = max(np.linalg.norm(fg[k, var] - fo[k, var]) / max(np.linalg.norm(fo[k, var]), 1e-300)
              for k in range(groups) for var in range(4) if np.linalg.norm(fo[k, var]) > 0)
    say("%s rho %.2e v %.2e sigma %.2e S %.2e wall %.2e" % (what, e_rho, e_v, e_s, e_S, e_f))
    errs = dict(rho=e_rho, v=e_v, sigma=e_s, S=e_S, wall=e_f)
    check_targets(errs, dict(rho=tf, v=tf, sigma=TOL_STRESS[storage], S=TOL_STRESS[storage],
                             wall=TOL_WALL[storage]), MISS_QUANT[storage], what)
    return errs


@pytest.mark.parametrize("model", [0, 1, 2, 3, 4])
def test_poiseuille_fp64_5000_steps(lbm, model):
    """Force-driven D2Q9 channel 64x32, FP64, 5000 steps: GPU vs oracle and
    vs the exact class-sum recurrence."""
    w = W.poiseuille(model=model)
    say("case poiseuille model", model)
    g = gpu_from(w, lbm)
    o = make_oracle(w)
    g.step(w.steps)
    o.step(w.steps)
    compare_all(g, o, W.F64, 2, "poiseuille")
    _, v = g.get_macro()
    assert rel_inf(v[0, 0, :, 0], channel_recurrence(w.ny, w.tau, 1e-6, w.steps)) < 1e-12
    bg, bo = g.force_balance(), o.force_balance()
    assert abs(bg[9]) < 1e-12 * bg[3] and abs(bg[22]) < 1e-12 * bg[21]
    assert rel_inf(bg[[0, 1, 3, 4, 6, 7, 18, 19, 21]], bo[[0, 1, 3, 4, 6, 7, 18, 19, 21]]) < 1e-12


STORAGES = [W.F64, W.F32, W.F16, W.BF16]


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("model", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_random_state_two_steps(lbm, lattice, model, storage):
    """Two steps (both A-A parities) from an arbitrary seeded state on a
    ragged lattice with plane walls, a moving wall, a solid body, LES and a
    non-unity dx, dt: every term of the step is exercised."""
    if lattice == W.D2Q9:
        nx, ny, nz = 37, 19, 1
        mask = W.cylinder_mask(nx, ny, 12.3, 9.1, 3.2)
        walls = ((1, 0, 1),)
    else:
        nx, ny, nz = 21, 13, 11
        mask = W.sphere_mask(nx, ny, nz, 9.4, 6.2, 5.1, 2.6)
        walls = ((1, 0, 1), (2, 2, 3))
    w = W.Workload("random", lattice, nx, ny, nz, 0.62, dx=0.5, dt=0.2, model=model, storage=storage,
                   body_force=(0.05, -0.02, 0.03), walls=walls, wall_velocity=((1, 0.08, 0.0, 0.03),),
                   obstacle=None, les_cs=0.1, groups=5)
    Q = 9 if lattice == W.D2Q9 else 19
    say("case random", lattice, model, storage)
    d0 = W.random_state(Q, nx, ny, nz, 2e-3, seed=17) * (1 - mask[None])
    g = gpu_from(w, lbm, init=False)
    g.add_solid_mask(mask, 4)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_state(quantize_state(d0, storage))  # the library stores the upload in its format
    low = storage in (W.F16, W.BF16)
    for k in range(2):
        g.step(1)
        if low:
            quantized_steps(o, storage, 1)
        else:
            o.step(1)
        st = rel_inf(g.get_state(), o.get_state())
        say("  step", k + 1, "state err %.2e" % st)
        check_targets(dict(state=st), TOL_FIELD[storage], MISS_QUANT[storage], "state")
        compare_all(g, o, storage, 5, "  step %d" % (k + 1))
    g.set_artefact(True)
    o.set_artefact(True)
    sg, Sg = g.stress()
    so, So = o.stress()
    check_targets(dict(sigma=rel_inf(sg, so), S=rel_inf(Sg, So)), TOL_STRESS[storage], MISS_QUANT[storage],
                  "with the artefact term")


def test_state_beyond_1gib_odd_steps_with_plain_loads(lbm):
    """FP32 duct with LES, 512x192x160 (15.7 M nodes, a 1.19 GB state): its
    odd steps read interior rows with plain loads (states beyond 1 GiB).  A
    3-step call (even, odd, then the diagnostic even step) against the
    oracle: state, stress and wall force at the FP32 tolerances."""
    import oracle
    oracle.threads(16)
    w = W.duct_les(nx=512, ny=192, nz=160)
    say("case plain loads 512x192x160")
    g = gpu_from(w, lbm)
    o = make_oracle(w)
    g.step(3)
    o.step(3)
    e_s = rel_inf(g.get_state(), o.get_state())
    say("  state %.2e" % e_s)
    assert e_s <= TOL_FIELD[W.F32]
    compare_all(g, o, W.F32, 4, "plain loads")


@pytest.mark.parametrize("storage", [W.F32, W.F64])
@pytest.mark.parametrize("nx", [256, 512, 768])
@pytest.mark.parametrize("case", ["walls", "periodic"])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_rows_staged_through_lds(lbm, lattice, case, nx, storage):
    """FP32 and FP64 odd steps stage the x-shifted directions of tiles of
    whole rows without boundary links through LDS (rows of 256 here); rows of
    512 and 768 take the unstaged buffer path, with the odd steps' tiles
    dealt to workgroups so that a row's tiles share an XCD (30 or 12 rows:
    whole groups of 8 rows and a remainder that keeps the identity).  Three-
    and four-step calls (staged odd steps between others, the last one with
    diagnostics) from a seeded state, with boundary rows (walls, a moving
    wall, a solid body) mixed in or a fully periodic box, against the
    oracle."""
    if lattice == W.D2Q9:
        ny, nz = 12, 1
        mask = W.cylinder_mask(nx, ny, 40.3, 6.1, 2.7)
        walls = ((1, 0, 1),)
    else:
        ny, nz = 6, 5
        mask = W.sphere_mask(nx, ny, nz, 60.4, 2.6, 2.1, 1.6)
        walls = ((1, 0, 1), (2, 2, 3))
    if case == "periodic":
        mask, walls = np.zeros_like(mask), ()
    w = W.Workload("lds_rows", lattice, nx, ny, nz, 0.62, dx=0.5, dt=0.2, model=W.GUO, storage=storage,
                   body_force=(0.05, -0.02, 0.03 if lattice == W.D3Q19 else 0.0), walls=walls,
                   wall_velocity=((1, 0.08, 0.0, 0.03),) if walls else (), les_cs=0.1, groups=5)
    Q = 9 if lattice == W.D2Q9 else 19
    say("case lds rows", lattice, case, nx, storage)
    d0 = W.random_state(Q, nx, ny, nz, 2e-3, seed=31) * (1 - mask[None])
    g = gpu_from(w, lbm, init=False)
    g.add_solid_mask(mask, 4)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_state(d0)
    for n in (3, 4):
        g.step(n)
        o.step(n)
        st = rel_inf(g.get_state(), o.get_state())
        say("  %d steps: state err %.2e" % (n, st))
        assert st <= TOL_FIELD[storage]
        if walls:
            compare_all(g, o, storage, 5, "  lds rows")


def test_couette_cylinder_fp32(lbm):
    """D2Q9 Couette + force + cylinder (reduced 128x32 version, 3000 steps),
    FP32 storage vs FP64 oracle; the momentum-flux correction vanishes."""
    w = W.couette_cylinder(nx=128, ny=32, r=6.0, cx=32.0, cy=16.0, steps=3000)
    g = gpu_from(w, lbm)
    o = make_oracle(w)
    g.step(w.steps)
    o.step(w.steps)
    compare_all(g, o, W.F32, 3, "couette")
    fw = g.wall_force()
    assert np.abs(fw[:, 1] - fw[:, 0]).max() < 1e-6 * np.abs(fw[:, 0]).max()


@pytest.mark.parametrize("storage", STORAGES)
def test_duct_les_small(lbm, storage):
    """Square duct with Smagorinsky closure and seeded +-1e-3 initial
    velocity (reduced 40x24x20), every storage format: 300 steps for FP64 and
    FP32; 30 steps for the 16-bit formats against the quantized oracle (over
    longer runs a single rounding that lands differently moves the two
    trajectories apart by a storage ulp, after which their rounding noise is
    independent and the comparison measures the format, which
    test_16bit_accuracy_vs_fp64 states)."""
    low = storage in (W.F16, W.BF16)
    w = W.duct_les(nx=40, ny=24, nz=20, steps=30 if low else 300)
    say("case duct", storage)
    g = gpu_from(w, lbm, storage=storage)
    o = make_oracle(w)
    g.step(w.steps)
    if low:
        o.set_state(quantize_state(o.get_state(), storage))
        quantized_steps(o, storage, w.steps)
    else:
        o.step(w.steps)
    compare_all(g, o, storage, 4, "duct %d" % storage)


# Recorded as not met against the unquantized FP64 oracle: the stress and
# strain rate under FP16 (the format's 11 significant bits; the quantized
# oracle, FP64 arithmetic with the same storage rounding, shows the same
# floor, so it is the format and not the kernel), and every result under
# BF16.  Bounds (regression checks) about 1.5 times the largest measured.
MISS_VS_FP64 = {W.F16: {"sigma": 1e-2, "S": 1e-2},
                W.BF16: {"rho": 8e-3, "v": 2e-2, "sigma": 1e-1, "S": 1e-1, "wall": 8e-3}}


@pytest.mark.parametrize("storage", [W.F16, W.BF16])
def test_16bit_accuracy_vs_fp64(lbm, storage):
    """Accuracy of 16-bit storage against the unquantized FP64 oracle
    (duct, 300 steps), at the 2e-3 target: FP16 meets it on density,
    velocity and wall force; its stress and strain rate, and BF16, are
    recorded as not met (MISS_VS_FP64)."""
    w = W.duct_les(nx=40, ny=24, nz=20, steps=300)
    g = gpu_from(w, lbm, storage=storage)
    o = make_oracle(w)
    g.step(w.steps)
    o.step(w.steps)
    rg, vg = g.get_macro()
    ro, vo = o.get_macro()
    sg, Sg = g.stress()
    so, So = o.stress()
    fg = g.wall_force()[:4, 0]
    fo = o.wall_force(4)[:, 0]
    e = dict(rho=np.abs(rg - ro).max(), v=rel_inf(vg, vo), sigma=rel_inf(sg, so), S=rel_inf(Sg, So),
             wall=np.linalg.norm(fg - fo) / np.linalg.norm(fo))
    say("16-bit %d vs FP64: %s" % (storage, {k: "%.2e" % v for k, v in e.items()}))
    check_targets(e, 2e-3, MISS_VS_FP64[storage], "storage %d vs FP64" % storage)


def test_duct_les_full_size_fp32(lbm):
    """256x128x128 duct with LES, FP32, in the bench's launch configuration:
    4 steps from the seeded start, full-field comparison."""
    w = W.duct_les()
    say("case duct full size")
    g = gpu_from(w, lbm)
    o = make_oracle(w)
    for k in range(2):
        g.step(2)
        o.step(2)
    compare_all(g, o, W.F32, 4, "duct full")
    bg = g.force_balance()
    assert np.abs(bg[9:12]).max() < 1e-4 * abs(bg[3])


def test_mhd_small(lbm):
    """Hartmann duct (reduced 12x16x12, 200 steps), FP32 and FP64 storage."""
    for storage in (W.F64, W.F32):
        w = W.hartmann_duct(nx=12, ny=16, nz=12, steps=200)
        say("case mhd", storage)
        g = gpu_from(w, lbm, storage=storage)
        o = make_oracle(w)
        g.step(w.steps)
        o.step(w.steps)
        compare_all(g, o, storage, 4, "mhd %d" % storage)
        Bg = g.get_field_B()
        _, _, Bo = o.get_macro(with_B=True)
        b0 = np.array(w.mhd[:3])[:, None, None, None]
        e_b = rel_inf(Bg - b0, Bo - b0)
        # the total Maxwell correction of a closed insulating duct is zero
        # (Eq. 36): compare it with the per-wall corrections it sums
        fo = o.wall_force(4)
        per_wall = np.abs(fo[:, 2] - fo[:, 0]).max()
        rg = g.force_balance()
        e_mx = np.abs(rg[12:15]).max() / per_wall
        say("  induced field B %.2e, total Maxwell correction / per wall %.2e" % (e_b, e_mx))
        assert e_b <= TOL_FIELD[storage]
        assert e_mx <= 1e-12


def test_determinism(lbm):
    w = W.duct_sphere(nx=32, ny=16, nz=16, r=3.0)
    outs = []
    for _ in range(2):
        g = gpu_from(w, lbm)
        g.step(37)
        outs.append((g.get_state(), g.wall_force(), g.force_balance()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


def test_unstable_state_is_reported(lbm):
    w = W.poiseuille(nx=8, ny=8)
    g = gpu_from(w, lbm, init=False)
    d = np.zeros((9, 1, 8, 8))
    d[3, 0, 4, 4] = np.nan
    g.set_state(d)
    with pytest.raises(lbm.LBMError) as ei:
        g.step(3)
    assert ei.value.code == lbm.LBM_EUNSTABLE


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("model", [0, 2, 4])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_halfstep_distribution(lbm, lattice, model, storage):
    """Half-step distribution (Eq. 27) and its stress (Eq. 28) after steps of
    both parities, from a seeded state, with a wall moving along its normal
    (the moving-wall term then changes the mass, which the library's
    reconstruction of f_rel must undo), a solid body and a per-node force."""
    if lattice == W.D2Q9:
        nx, ny, nz = 64, 19, 1
        mask = W.cylinder_mask(nx, ny, 12.3, 9.1, 3.2)
        walls = ((1, 0, 1),)
    else:
        nx, ny, nz = 21, 13, 11
        mask = W.sphere_mask(nx, ny, nz, 9.4, 6.2, 5.1, 2.6)
        walls = ((1, 0, 1), (2, 2, 3))
    w = W.Workload("half", lattice, nx, ny, nz, 0.7, dx=0.5, dt=0.2, model=model, storage=storage,
                   walls=walls, wall_velocity=((1, 0.08, -0.05, 0.03),), groups=5)
    Q = 9 if lattice == W.D2Q9 else 19
    say("case halfstep", lattice, model, storage)
    d0 = W.random_state(Q, nx, ny, nz, 2e-3, seed=21) * (1 - mask[None])
    af = W.force_field(nx, ny, nz, base=(0.05, -0.02, 0.03), amp=0.5, seed=22)
    if lattice == W.D2Q9:
        af[2] = 0.0
    import torch
    at = torch.from_numpy(af.astype(np.float32)).cuda()
    torch.cuda.synchronize()
    g = gpu_from(w, lbm, init=False)
    g.add_solid_mask(mask, 4)
    g.set_body_force_field(at.data_ptr())
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_body_force_field(af.astype(np.float32).astype(np.float64))
    o.set_state(quantize_state(d0, storage))
    tf, ts = TOL_FIELD[storage], TOL_STRESS[storage]
    for k in range(2):
        g.step(1)
        o.step(1)
        fg, rg, ug, sg = g.halfstep()
        fo, ro, uo, so = o.halfstep()
        e = dict(f=rel_inf(fg, fo), rho=np.abs(rg - ro).max(), u=rel_inf(ug, uo), sigma=rel_inf(sg, so))
        say("  step %d: %s" % (k + 1, {n: "%.2e" % v for n, v in e.items()}))
        assert e["f"] <= tf and e["rho"] <= tf and e["u"] <= tf and e["sigma"] <= ts


def test_halfstep_mhd(lbm):
    """Hartmann duct after 200 and 201 steps (both parities; from rest the
    velocity needs some steps to rise well above the rounding of the oracle's
    magnetic equilibrium terms, which it keeps inside its deviations)."""
    for storage in (W.F64, W.F32):
        w = W.hartmann_duct(nx=12, ny=16, nz=12, steps=0)
        say("case halfstep mhd", storage)
        g = gpu_from(w, lbm, storage=storage)
        o = make_oracle(w)
        for k in range(2):
            g.step(200 if k == 0 else 1)
            o.step(200 if k == 0 else 1)
            fg, rg, ug, sg = g.halfstep()
            fo, ro, uo, so = o.halfstep()
            e = dict(f=rel_inf(fg, fo), rho=np.abs(rg - ro).max(), u=rel_inf(ug, uo), sigma=rel_inf(sg, so))
            say("  %s" % {n: "%.2e" % v for n, v in e.items()})
            assert e["f"] <= TOL_FIELD[storage] and e["rho"] <= TOL_FIELD[storage]
            assert e["u"] <= TOL_FIELD[storage] and e["sigma"] <= TOL_STRESS[storage]


@pytest.mark.parametrize("curved", [False, True])
def test_halfstep_into_device_buffers_equals_host_outputs(lbm, curved):
    """lbm_halfstep_device writes the same values (bit for bit) into caller
    device buffers as lbm_halfstep does into host buffers: a duct with a
    sphere, halfway or with interpolated walls, after a 7-step call; with
    some outputs left NULL."""
    import torch
    w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7)
    w.curved = curved
    say("case halfstep device", curved)
    g = gpu_from(w, lbm)
    g.step(7)
    fh, rh, uh, sh = g.halfstep()
    dev = dict(dtype=torch.float64, device="cuda")
    fb = torch.full(fh.shape, 7.0, **dev)
    rb = torch.full(rh.shape, 7.0, **dev)
    ub = torch.full(uh.shape, 7.0, **dev)
    sb = torch.full(sh.shape, 7.0, **dev)
    torch.cuda.synchronize()
    g.halfstep_device(fb.data_ptr(), rb.data_ptr(), ub.data_ptr(), sb.data_ptr())
    torch.cuda.synchronize()
    for a, b in ((fb, fh), (rb, rh), (ub, uh), (sb, sh)):
        assert np.array_equal(a.cpu().numpy(), b)
    sb.fill_(7.0)
    rb.fill_(7.0)
    torch.cuda.synchronize()
    g.halfstep_device(None, None, None, sb.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(sb.cpu().numpy(), sh)
    assert float(rb.cpu().max()) == 7.0  # left alone


def test_halfstep_needs_a_step(lbm):
    w = W.poiseuille(nx=8, ny=8)
    g = gpu_from(w, lbm)
    with pytest.raises(lbm.LBMError) as ei:
        g.halfstep()
    assert ei.value.code == lbm.LBM_ESTATE
    with pytest.raises(lbm.LBMError) as ei:
        g.halfstep_device(None, None, None, None)
    assert ei.value.code == lbm.LBM_ESTATE


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("model", [0, 2, 4])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_stokes_equilibrium_and_darcy_resistance(lbm, lattice, model, storage):
    """Two steps with the Stokes form of the equilibrium and a porous
    resistance (text after Eq. 11), from a seeded state with walls, a moving
    wall and a solid body; then the half-step stress."""
    if lattice == W.D2Q9:
        nx, ny, nz = 64, 19, 1
        mask = W.cylinder_mask(nx, ny, 12.3, 9.1, 3.2)
        walls = ((1, 0, 1),)
    else:
        nx, ny, nz = 21, 13, 11
        mask = W.sphere_mask(nx, ny, nz, 9.4, 6.2, 5.1, 2.6)
        walls = ((1, 0, 1), (2, 2, 3))
    w = W.Workload("stokes", lattice, nx, ny, nz, 0.65, dx=0.5, dt=0.2, model=model, storage=storage,
                   body_force=(0.05, -0.02, 0.03), walls=walls, wall_velocity=((1, 0.08, 0.0, 0.03),),
                   stokes=True, darcy=0.7, groups=5)
    Q = 9 if lattice == W.D2Q9 else 19
    say("case stokes+darcy", lattice, model, storage)
    d0 = W.random_state(Q, nx, ny, nz, 2e-3, seed=31) * (1 - mask[None])
    g = gpu_from(w, lbm, init=False)
    g.add_solid_mask(mask, 4)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_state(quantize_state(d0, storage))
    for k in range(2):
        g.step(1)
        o.step(1)
        assert rel_inf(g.get_state(), o.get_state()) <= TOL_FIELD[storage]
        compare_all(g, o, storage, 5, "  step %d" % (k + 1))
    _, _, _, sg = g.halfstep()
    _, _, _, so = o.halfstep()
    assert rel_inf(sg, so) <= TOL_STRESS[storage]
    rg, ro = g.force_balance(), o.force_balance()
    assert np.abs(rg[3:6] - ro[3:6]).max() <= TOL_WALL[storage] * np.abs(ro[3:6]).max()
    # the artefact term of Eq. (9) under the Stokes form (only -tau Theta)
    g.set_artefact(True)
    o.set_artefact(True)
    sg, Sg = g.stress()
    so, So = o.stress()
    e_s, e_S = rel_inf(sg, so), rel_inf(Sg, So)
    say("  with the artefact term: sigma %.2e S %.2e" % (e_s, e_S))
    assert e_s <= TOL_STRESS[storage] and e_S <= TOL_STRESS[storage]
