"""cmlbm_step_reduce (one step whose kernel also forms the FP64 reductions of
the state it reads) against cmlbm_reduce followed by cmlbm_step on a twin
lattice: the same state afterwards (to a unit or two in the last place of the
stored format: the compiler may contract the two kernels' arithmetic
differently), the same counts, and sums that agree to the rounding of the
per-cell values of the step's arithmetic."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = {"mass": 0, "momx": 1, "momy": 2, "momz": 3, "ke": 4, "umax": 5, "nonfinite": 6, "fluid": 7, "u2": 9}
# D3Q27 weights by class (|c|^2 = 0, 1, 2, 3) in the export order of cmlbm_populations
WGT = None


def weights():
    import oracle as O
    return O.constants()[3]


def ulp(h, storage):
    """Two units in the last place of the stored value h = f - w rho0 (FP64 and
    FP32 store h itself; FP16 stores 256 h; BF16 h with 8 significant bits),
    plus the FP32 spacing of f below 1 for the 16-bit formats, whose stored
    values are decoded exactly."""
    a = np.abs(h)
    if storage == "fp64":
        return 2 * np.spacing(np.maximum(a, 1.0))
    if storage == "fp32":
        return 2 * np.spacing(np.maximum(a, 0.5).astype(np.float32)).astype(np.float64)
    if storage == "fp16":
        return np.spacing((a * 256).astype(np.float16)).astype(np.float64) / 256 + 1e-12
    return np.ldexp(1.0, np.floor(np.log2(np.maximum(a, 2.0 ** -126))).astype(np.int64) - 7) + 1e-12


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def pair(storage, nx, ny, nz, nbatch=1, wall=(0, 0, 0), solid=None, field=None, steps=3, seed=5, stochastic=False):
    from paper_1905_10182_amd import Lattice
    g = W.generator(seed)
    u = g.uniform(-0.04, 0.04, size=(3, nbatch, nz, ny, nx))
    rho = 1.0 + g.uniform(-1e-3, 1e-3, size=(nbatch, nz, ny, nx))
    lats = []
    for fused in (True, False):
        lat = Lattice(nx, ny, nz, nbatch=nbatch, tau=0.6, storage=storage, wall=wall, solid=solid is not None,
                      stochastic=stochastic, fused_reduce=fused, device="cuda:0")
        if solid is not None:
            lat.set_solid(solid)
        if field is not None:
            lat.set_force("field", field=field)
        lat.init(rho, u)
        lat.step(steps)
        lats.append(lat)
    return lats


def check(torch, a, b, storage, nsteps=2):
    """a: fused lattice, b: twin.  nsteps of step_reduce against reduce + step."""
    global WGT
    if WGT is None:
        WGT = np.asarray(weights(), np.float64)
    for k in range(nsteps):
        ref = b.reduce()
        b.step(1)
        got = a.step_reduce()
        assert np.array_equal(got[:, KEYS["fluid"]], ref[:, KEYS["fluid"]])
        assert np.all(got[:, KEYS["nonfinite"]] == 0)
        # sums over cells: per-cell FP32 rounding averages out; the maximum is one cell's value
        rtol = 1e-13 if storage == "fp64" else 2e-6
        n = ref[:, KEYS["fluid"]]
        for key in ("ke", "u2"):
            np.testing.assert_allclose(got[:, KEYS[key]], ref[:, KEYS[key]], rtol=rtol, atol=0)
        np.testing.assert_allclose(got[:, KEYS["umax"]], ref[:, KEYS["umax"]], rtol=1e-13 if storage == "fp64" else 1e-5)
        # mass and momentum sums: per-cell rounding of O(1) quantities
        atol = (1e-14 if storage == "fp64" else 2e-7) * n
        for key in ("mass", "momx", "momy", "momz"):
            np.testing.assert_allclose(got[:, KEYS[key]], ref[:, KEYS[key]], rtol=0, atol=atol.max())
        log(f"  step {k}: ke {got[0, 4]:.10e} vs {ref[0, 4]:.10e}")
        # the compiler contracts the two kernels' arithmetic differently, so the
        # states agree to the last unit of the arithmetic, not bit for bit
        pa, pb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
        d = np.abs(pa - pb)
        h = pb - WGT.reshape((27,) + (1,) * (pb.ndim - 1))
        log(f"  state: {np.mean(d == 0):.4f} of populations bitwise equal, max |diff| {d.max():.2e}")
        assert np.all(d <= ulp(h, storage)), "fused step changed the state beyond one unit in the last place"
    assert a.time == b.time


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("nx", [40, 37, 128])
def test_fused_reduce_periodic(torch, storage, nx):
    """Ragged rows (40: one partial wave per row, two cells per lane for 16-bit;
    37: odd, one cell per lane; 128: a row of exactly one or two waves)."""
    log(f"{storage} fused reductions, {nx}x12x10 periodic")
    a, b = pair(storage, nx, 12, 10)
    check(torch, a, b, storage)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [40, 37])
def test_fused_reduce_stochastic_rounding(torch, storage, nx):
    """16-bit storage with stochastic rounding: the fused kernel draws the same
    counter-based bits for each (cell, step) as the plain one."""
    log(f"{storage} stochastic rounding, fused reductions, {nx}x12x10")
    a, b = pair(storage, nx, 12, 10, stochastic=True)
    check(torch, a, b, storage)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_fused_reduce_walls_solid_field_batch(torch, storage):
    """Walls on two axes, solid nodes (their lanes stay for the wave sum but
    neither contribute nor store), a per-cell force field and a batch of two
    lattices whose partial sums are kept apart."""
    log(f"{storage} fused reductions, 70x13x9 x2, walls, solids, field force")
    nb, nz, ny, nx = 2, 9, 13, 70
    g = W.generator(11)
    solid = (g.random((nb, nz, ny, nx)) < 0.08).astype(np.uint8)
    field = g.uniform(-1e-5, 1e-5, size=(3, nb, nz, ny, nx))
    a, b = pair(storage, nx, ny, nz, nbatch=nb, wall=(0, 1, 1), solid=solid, field=field)
    check(torch, a, b, storage)
    got = a.step_reduce()
    assert np.array_equal(got[:, KEYS["fluid"]], (1 - solid).reshape(nb, -1).sum(1).astype(float))


def test_fused_reduce_reproducible_and_needs_flag(torch):
    from paper_1905_10182_amd import Lattice
    from paper_1905_10182_amd.cmlbm import CmlbmError
    wl = W.taylor_green(32, seed=1)
    outs = []
    for _ in range(2):
        lat = Lattice(32, 32, 32, tau=wl["tau"], storage="fp32", fused_reduce=True, device="cuda:0")
        lat.init(wl["rho"], wl["u"])
        outs.append(np.stack([lat.step_reduce() for _ in range(3)]))
    assert np.array_equal(outs[0], outs[1])
    plain = Lattice(32, 32, 32, tau=wl["tau"], storage="fp32", device="cuda:0")
    plain.init(wl["rho"], wl["u"])
    with pytest.raises(CmlbmError, match="ESTATE"):
        plain.step_reduce()


def test_fused_reduce_bench_size(torch):
    """The benchmark's fused-reduction leg (FP32 TGV 256^3, 1024-thread
    workgroups): step_reduce's sums of the state against reduce() of the same
    state."""
    from paper_1905_10182_amd import Lattice
    wl = W.taylor_green(256, seed=1)
    lat = Lattice(256, 256, 256, tau=wl["tau"], storage="fp32", fused_reduce=True, device="cuda:0")
    lat.init(wl["rho"], wl["u"])
    del wl
    lat.step(3)
    ref = lat.reduce()
    got = lat.step_reduce()
    log(f"  fp32 256^3: ke {got[0, 4]:.10e} vs {ref[0, 4]:.10e}, mass {got[0, 0]:.10e} vs {ref[0, 0]:.10e}")
    assert got[0, KEYS["fluid"]] == ref[0, KEYS["fluid"]] == 256 ** 3
    for key in ("ke", "u2"):
        assert abs(got[0, KEYS[key]] / ref[0, KEYS[key]] - 1) < 2e-6
    assert abs(got[0, KEYS["umax"]] / ref[0, KEYS["umax"]] - 1) < 1e-5
    n = 256 ** 3
    for key in ("mass", "momx", "momy", "momz"):
        assert abs(got[0, KEYS[key]] - ref[0, KEYS[key]]) < 2e-7 * n
