"""Full-size parity on the 512^3 large-shot workload, in the launch
configuration the benchmark times (automatic kernel choice).

(a) the first 40 steps of the full grid against the FP64 oracle
    (relative L2 <= 1e-5 on the field and the traces), and the whole
    1000-step shot against the oracle's whole 1000-step run (the error
    accumulated over the shot: measured 3.8e-6 on the field and 1.7e-6 on
    the traces, within the plain FP32 path's bound of 1e-5); the same run
    of the oracle also checks the u-and-change 16-bit forms over the whole
    shot against the bounds proposed for 16-bit storage;
(b) the whole 1000-step shot, checked at sampled cells: the oracle
    evaluates step 1000 point by point from the GPU's own u^999, u^998
    and k, which isolates one step's FP32 rounding at full size;
(c) the same sampled check on the paper's largest and smallest Table 2 grids;
(d) one step on the largest plane one buffer resource addresses (2 GiB)."""
import numpy as np
import pytest
import torch

from paper_2204_03775_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def shot():
    return inputs.large_shot()


@pytest.fixture(scope="module")
def prop(wave_mod, shot):
    p = shot
    pr = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    pr.record(p.nt)
    yield pr
    pr.close()


def test_first_steps_full_grid(wave_mod, oracle_lib, shot, prop):
    p, nt = shot, 40
    print(f"case: 512^3 full grid, {nt} steps, config {prop.config()}", flush=True)
    prop.reset()
    prop.run(nt, torch.tensor(p.s[:nt], dtype=torch.float32, device="cuda"))
    prop.sync()
    cur, _, n = prop.fields()
    got = prop.interior(cur).cpu().numpy()
    tr = prop.traces[:nt, :prop.nrec].cpu().numpy()
    ref, _, rtr = oracle_lib.run(p.k64(), p.h, nt, s=p.s, src=p.src, rec=p.rec,
                                 sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    e_f, e_t = rel(got, ref), rel(tr, rtr)
    print(f"rel-L2 field {e_f:.3e} traces {e_t:.3e}")
    assert n == nt
    assert e_f <= 1e-5 and e_t <= 1e-5


@pytest.fixture(scope="module")
def whole_shot_reference(request, oracle_lib, shot):
    # the FP64 oracle's own 1000-step run of the benchmark's shot (about two
    # minutes on 16 host cores, in segments with a progress line each, shown
    # past pytest's output capture)
    p = shot
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def progress(done, nt, sec):
        with capman.global_and_fixture_disabled():
            print(f"  oracle 512^3: {done}/{nt} steps, {sec:.0f} s", flush=True)

    ref, _, rtr, sec = oracle_lib.run_segments(p.k64(), p.h, p.nt, 200, s=p.s, src=p.src, rec=p.rec,
                                               sponge_width=p.sponge_width,
                                               sponge_alpha=p.sponge_alpha, progress=progress)
    return ref, rtr, sec


@pytest.mark.timeout(1200)
def test_full_shot_against_oracle(wave_mod, shot, prop, whole_shot_reference):
    # The benchmark's shot in full: 1000 steps of 512^3 (Eq. 2 and Algorithm 1
    # at the step count of the paper's Table 2 runs) against the FP64
    # oracle's own 1000-step run, on the final field and all 256,000 trace
    # values.
    p = shot
    print(f"case: 512^3 full shot vs oracle, {p.nt} steps, config {prop.config()}", flush=True)
    prop.reset()
    prop.run(p.nt, torch.tensor(p.s, dtype=torch.float32, device="cuda"))
    prop.sync()
    cur, _, n = prop.fields()
    got = prop.interior(cur).cpu().numpy()
    tr = prop.traces[:, :prop.nrec].cpu().numpy()
    assert n == p.nt
    ref, rtr, sec = whole_shot_reference
    e_f, e_t = rel(got, ref), rel(tr, rtr)
    print(f"  512^3 x {p.nt}: rel-L2 field {e_f:.3e} traces {e_t:.3e} (oracle {sec:.0f} s, "
          f"{p.points * p.nt / sec / 1e9:.2f} Gpts/s)", flush=True)
    assert e_f <= 1e-5 and e_t <= 1e-5


# the u-and-change 16-bit forms over the whole shot, against the bounds
# proposed for 16-bit storage (measured 4.1e-3 / 1.8e-3 for FP16, 3.6e-2 /
# 1.6e-2 for BF16, field / traces); the two-level forms miss these bounds
# and are regression-pinned on the 128^3 crop instead
WHOLE_SHOT_BOUNDS = {"f16uv": 5e-3, "bf16uv": 5e-2}


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("dtype", sorted(WHOLE_SHOT_BOUNDS))
def test_storage_forms_full_shot_against_oracle(wave_mod, shot, whole_shot_reference, dtype):
    p = shot
    pr = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dtype)
    pr.record(p.nt)
    print(f"case: 512^3 full shot, {dtype}, config {pr.config()}", flush=True)
    pr.run(p.nt, torch.tensor(p.s, dtype=torch.float32, device="cuda"))
    pr.sync()
    got = pr.export(0).cpu().numpy()
    tr = pr.traces[:, :pr.nrec].cpu().numpy()
    n = pr.fields()[2]
    pr.close()
    assert n == p.nt
    ref, rtr, _ = whole_shot_reference
    e_f, e_t = rel(got, ref), rel(tr, rtr)
    print(f"  {dtype} 512^3 x {p.nt}: rel-L2 field {e_f:.3e} traces {e_t:.3e}", flush=True)
    assert e_f <= WHOLE_SHOT_BOUNDS[dtype] and e_t <= WHOLE_SHOT_BOUNDS[dtype]


def _sample_points(p, rng):
    nz, ny, nx = p.shape
    pts = [rng.integers(0, [nz, ny, nx], size=(16000, 3))]
    # tile, chunk and sponge boundaries, faces and the source neighbourhood
    edges_x = sorted({0, 1, 2, 3, nx - 1, nx - 4} | {e + d for e in range(64, nx, 64)
                                                     for d in (-1, 0)} | {19, 20})
    edges_y = sorted({0, 3, ny - 1, ny - 4} | {e + d for e in range(8, ny, 8) for d in (-1, 0)})
    edges_z = sorted({0, 3, nz - 1, nz - 4, 19, 20} | {e + d for e in range(32, nz, 32)
                                                       for d in (-1, 0)})
    for _ in range(4000):
        pts.append(np.array([[rng.choice(edges_z), rng.choice(edges_y), rng.choice(edges_x)]]))
    sz, sy, sx = p.src
    for dz in range(-4, 5):
        for dy in range(-4, 5):
            for dx in range(-4, 5):
                pts.append(np.array([[sz + dz, sy + dy, sx + dx]]))
    pts.append(np.asarray(p.rec))
    pts = np.unique(np.concatenate(pts).astype(np.int32), axis=0)
    return pts


def test_full_shot_sampled(wave_mod, oracle_lib, shot, prop):
    p = shot
    print(f"case: 512^3 full shot, {p.nt} steps, config {prop.config()}", flush=True)
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    prop.reset()
    prop.run(p.nt - 1, s)
    prop.sync()
    cur, prev, _ = prop.fields()
    u_cur = prop.interior(cur).cpu().numpy()
    u_prev = prop.interior(prev).cpu().numpy()
    prop.run(1, s[p.nt - 1:])
    prop.sync()
    new, _, n = prop.fields()
    u_new = prop.interior(new).cpu().numpy()
    tr = prop.traces[:, :prop.nrec].cpu().numpy()
    assert n == p.nt
    assert np.isfinite(u_new).all() and np.isfinite(tr).all()
    assert np.abs(tr).max() > 0
    # the last trace row is u^{1000} at the receivers
    rz, ry, rx = np.asarray(p.rec).T
    assert np.array_equal(tr[-1], u_new[rz, ry, rx])

    pts = _sample_points(p, np.random.default_rng(77))
    k32 = p.k32()
    ref = oracle_lib.step_points(k32, u_cur, u_prev, p.h, pts, sponge_width=p.sponge_width,
                                 sponge_alpha=p.sponge_alpha, src=p.src,
                                 src_value=float(np.float32(p.s[p.nt - 1])))
    got = u_new[pts[:, 0], pts[:, 1], pts[:, 2]].astype(np.float64)
    scale = np.abs(u_cur).max()
    err = np.abs(got - ref)
    print(f"{len(pts)} points: max |diff| {err.max():.3e} (field max {scale:.3e}), "
          f"rel-L2 {rel(got, ref):.3e}")
    assert err.max() <= 1e-6 * scale
    assert rel(got, ref) <= 1e-6


@pytest.mark.parametrize("dtype,eps", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_full_shot_sampled_16bit(wave_mod, oracle_lib, shot, dtype, eps):
    # the two-level 16-bit forms at full size, in the benchmark's launch
    # configuration: step 1000 evaluated by the oracle at sampled cells from
    # the GPU's decoded u^999, u^998.  The GPU also rounds k (relative eps)
    # and the stored u^1000 (eps / 2 relative): with |k lap| <= 4 M and
    # |u^1000| <= 7 M (M = max |u^999|, |u^998|) the difference stays below
    # 8 eps M.
    p = shot
    pr = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dtype)
    print(f"case: 512^3 full shot {dtype}, config {pr.config()}", flush=True)
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    pr.run(p.nt - 1, s)
    u_cur = pr.export(0).cpu().numpy()
    u_prev = pr.export(1).cpu().numpy()
    pr.run(1, s[p.nt - 1:])
    u_new = pr.export(0).cpu().numpy()
    pr.sync()
    _, _, n = pr.fields()
    pr.close()
    assert n == p.nt and np.isfinite(u_new).all()
    pts = _sample_points(p, np.random.default_rng(78))
    ref = oracle_lib.step_points(p.k32(), u_cur, u_prev, p.h, pts, sponge_width=p.sponge_width,
                                 sponge_alpha=p.sponge_alpha, src=p.src,
                                 src_value=float(np.float32(p.s[p.nt - 1])))
    got = u_new[pts[:, 0], pts[:, 1], pts[:, 2]].astype(np.float64)
    M = max(np.abs(u_cur).max(), np.abs(u_prev).max())
    err = np.abs(got - ref).max()
    print(f"{len(pts)} points: max |diff| {err:.3e} = {err / (eps * M):.2f} eps M")
    assert err <= 8 * eps * M


@pytest.mark.parametrize("shape", [(755, 994, 1000), (200, 200, 1000)], ids=lambda s: "x".join(map(str, s)))
def test_paper_shape_sampled(wave_mod, oracle_lib, shape):
    # The paper's largest and smallest Table 2 grids, in the launch
    # configuration the paper-shape leg times.  755 x 994 x 1000: nx is not
    # a multiple of 4 (each row ends in a ragged 4-cell group stored whole)
    # and the plan makes three rounds of work-groups.  200 x 200 x 1000: one
    # 256 x 8 tile across, 50 of each row's 64 lanes in the grid, ten
    # z-chunks.  Step nt is evaluated by the oracle at sampled cells from the
    # GPU's own u^{nt-1}, u^{nt-2}; every cell past nx (ghost and row
    # padding) must still be zero.
    nt = 60
    p = inputs.paper_shape(nt, *shape)
    nz, ny, nx = p.shape
    kval = np.float32((np.float64(1500.0) * p.dt) ** 2)
    k = torch.full((1, 1, 1), float(kval), dtype=torch.float32, device="cuda").expand(nz, ny, nx)
    pr = wave_mod.Propagator(nx, ny, nz, p.h, k, src=p.src, rec=p.rec)
    del k
    pr.record(nt)
    variant, zc, _ = pr.config()
    tile_x, tile_y = (int(v) for v in wave_mod.wave_variant_name(variant)[1:].split("_")[0].split("x"))
    print(f"case: {nx}x{ny}x{nz}, {nt} steps, config {pr.config()}", flush=True)
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    pr.run(nt - 1, s)
    pr.sync()
    cur, prev, _ = pr.fields()
    u_cur = pr.interior(cur).cpu().numpy()
    u_prev = pr.interior(prev).cpu().numpy()
    pr.run(1, s[nt - 1:])
    pr.sync()
    new, _, n = pr.fields()
    assert n == nt
    x0 = pr.layout.x_offset
    for b in pr.buf:
        assert torch.count_nonzero(pr.padded(b)[:, :, x0 + nx:]).item() == 0
        assert torch.count_nonzero(pr.padded(b)[:, :, :x0]).item() == 0
    u_new = pr.interior(new).cpu().numpy()
    tr = pr.traces[:, :pr.nrec].cpu().numpy()
    assert np.isfinite(tr).all() and np.abs(tr).max() > 0
    rz, ry, rx = np.asarray(p.rec).T
    assert np.array_equal(tr[-1], u_new[rz, ry, rx])
    pr.close()

    rng = np.random.default_rng(755)
    pts = [rng.integers(0, [nz, ny, nx], size=(20000, 3))]
    edges_x = sorted({0, 1, 3, 4, nx - 5, nx - 4, nx - 3, nx - 2, nx - 1} |
                     {e + d for e in range(tile_x, nx, tile_x) for d in (-1, 0)})
    edges_y = sorted({0, 3, ny - 1, ny - 4} | {e + d for e in range(tile_y, ny, tile_y) for d in (-1, 0)})
    edges_z = sorted({0, 3, nz - 1, nz - 4} | {e + d for e in range(zc, nz, zc) for d in (-4, -1, 0, 3)})
    for _ in range(4000):
        pts.append(np.array([[rng.choice(edges_z), rng.choice(edges_y), rng.choice(edges_x)]]))
    sz, sy, sx = p.src
    pts.append(np.array([[sz + dz, sy + dy, sx + dx] for dz in range(-4, 5) for dy in range(-4, 5)
                         for dx in range(-4, 5)]))
    pts = np.unique(np.concatenate(pts).astype(np.int32), axis=0)
    k32 = np.broadcast_to(kval, (nz, ny, nx))
    ref = oracle_lib.step_points(k32, u_cur, u_prev, p.h, pts, src=p.src,
                                 src_value=float(np.float32(p.s[nt - 1])))
    got = u_new[pts[:, 0], pts[:, 1], pts[:, 2]].astype(np.float64)
    scale = np.abs(u_cur).max()
    err = np.abs(got - ref)
    print(f"{len(pts)} points: max |diff| {err.max():.3e} (field max {scale:.3e}), rel-L2 {rel(got, ref):.3e}")
    assert err.max() <= 1e-6 * scale
    assert rel(got, ref) <= 1e-6


def test_maximum_plane_sampled(wave_mod, oracle_lib):
    # The largest FP32 plane one buffer resource addresses (2 GiB): 23000 x
    # 23000 cells plus ghosts and row padding, two planes deep.  Seeded
    # random fields fill the whole grid, so every in-plane byte offset the
    # kernel forms (up to 2.1e9) carries a value.  One step is checked at
    # the corners, the source and an interior window by the oracle's
    # pointwise step on crops of u^n, u^{n-1} (cells at least 4 from a crop
    # edge that is not a grid edge, so the crop's zero surround is never
    # read).  FP32 rounding of the update of values |u| <= M stays far
    # below 32 * 2^-24 * M; an offset error would be of order M.
    nx = ny = 23000
    nz = 2
    L = wave_mod.wave_layout(nx, ny, nz)
    assert 0.95 * 2 ** 31 < 4 * L.plane < 2 ** 31
    with pytest.raises(wave_mod.WaveError):
        wave_mod.wave_layout(nx + 1024, ny, nz)  # a plane past 2 GiB
    p = inputs.paper_shape(2, nx, ny, nz)
    kval = np.float32((np.float64(1500.0) * p.dt) ** 2)
    k = torch.full((1, 1, 1), float(kval), dtype=torch.float32, device="cuda").expand(nz, ny, nx)
    pr = wave_mod.Propagator(nx, ny, nz, p.h, k, src=p.src, rec=[(0, 0, 0), (nz - 1, ny - 1, nx - 1)])
    del k
    pr.record(1)
    print(f"case: maximum plane {nx}x{ny}x{nz}, config {pr.config()}", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(2300)
    for b in pr.buf:
        pr.interior(b).copy_(torch.rand((nz, ny, nx), generator=gen, device="cuda") - 0.5)
    cur, prev, _ = pr.fields()
    sy, sx = p.src[1], p.src[2]
    windows = [(0, 48, 0, 48), (0, 48, nx - 48, nx), (ny - 48, ny, 0, 48), (ny - 48, ny, nx - 48, nx),
               (sy - 24, sy + 24, sx - 24, sx + 24), (9001, 9049, 15007, 15055)]
    crops = [(pr.interior(cur)[:, y0:y1, x0:x1].cpu().numpy(), pr.interior(prev)[:, y0:y1, x0:x1].cpu().numpy())
             for y0, y1, x0, x1 in windows]
    s = torch.tensor([np.float32(p.s[0])], dtype=torch.float32, device="cuda")
    pr.run(1, s)
    pr.sync()
    new, _, n = pr.fields()
    assert n == 1
    x0p = pr.layout.x_offset
    tail = pr.padded(new)[:, :, x0p + nx:]
    assert torch.count_nonzero(tail).item() == 0  # row padding past the last column
    tr = pr.traces[0, :2].cpu().numpy()
    errs, refs = [], []
    M = 0.0
    for (y0, y1, x0, x1), (uc, up) in zip(windows, crops):
        got_all = pr.interior(new)[:, y0:y1, x0:x1].cpu().numpy()
        lo_y = 0 if y0 == 0 else 4
        hi_y = (y1 - y0) if y1 == ny else (y1 - y0) - 4
        lo_x = 0 if x0 == 0 else 4
        hi_x = (x1 - x0) if x1 == nx else (x1 - x0) - 4
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(lo_y, hi_y), np.arange(lo_x, hi_x), indexing="ij")
        pts = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], axis=1).astype(np.int32)
        src = None
        if y0 <= sy < y1 and x0 <= sx < x1:
            src = (p.src[0], sy - y0, sx - x0)
        kc = np.broadcast_to(kval, uc.shape)
        ref = oracle_lib.step_points(kc, uc, up, p.h, pts, src=src, src_value=float(np.float32(p.s[0])))
        got = got_all[pts[:, 0], pts[:, 1], pts[:, 2]].astype(np.float64)
        errs.append(np.abs(got - ref))
        refs.append(ref)
        M = max(M, float(np.abs(uc).max()), float(np.abs(up).max()))
        if (y0, x0) == (0, 0):
            assert tr[0] == got_all[0, 0, 0]
        if (y1, x1) == (ny, nx):
            assert tr[1] == got_all[nz - 1, -1, -1]
    pr.close()
    err = np.concatenate(errs)
    ref = np.concatenate(refs)
    eps = 2.0 ** -24
    print(f"{err.size} points: max |diff| {err.max():.3e} = {err.max() / (eps * M):.2f} eps M", flush=True)
    assert err.max() <= 32 * eps * M
    assert np.linalg.norm(err) / np.linalg.norm(ref) <= 1e-6
