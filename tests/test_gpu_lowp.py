"""Reduced-precision storage (FP16 / BF16 fields, FP32 arithmetic).

Exact checks:
  - every tiled kernel and z-chunk agrees bit for bit with the naive
    kernel (same decode, arithmetic, encode and scale choice);
  - the per-level power-of-two scaling makes the scheme exactly
    equivariant: multiplying the source by 2^j leaves every stored bit
    unchanged and multiplies every decoded field value and trace by 2^j,
    bit for bit wherever the decoded value is an FP32 normal (BF16 keeps
    FP32's exponent range, so decoding can land in the subnormals, where a
    power-of-two scaling is not exact; there the values agree to FLT_MIN);
  - the stored bits, level exponent and traces equal, bit for bit, those of
    the CPU emulation of the scheme in oracle/oracle16.c (pinned on its own
    against numpy's float16, nearest-even bfloat16 rounding and the FP64
    update of its decoded inputs), on a ragged grid and on the 128^3 crop.
Accuracy against the FP64 oracle (relative L2 on field and traces), bounds
stated per format from the formats' unit roundoff (FP16 2^-11, BF16 2^-8)
and the measured error growth:
  - 64^3 parity workload, 100 steps;
  - 128^3 crop of the large-shot model with its own sponge, 500 steps."""
import numpy as np
import pytest
import torch

from paper_2204_03775_amd import inputs

pytestmark = pytest.mark.gpu

# Bounds (relative L2 against the FP64 oracle).  u-and-change storage keeps
# the step change d^n to its own precision; measured f16uv 8.6e-4 (64^3),
# 3.1e-3 / 1.7e-3 (crop field / traces); bf16uv 8.2e-3, 2.5e-2 / 1.4e-2.
# Their bounds are about twice the measured values and within the ones
# proposed for reduced-precision storage (FP16 5e-3, BF16 5e-2).
# The two-level forms do NOT meet those proposed bounds on the crop: at this
# Courant number the per-step change u^n - u^{n-1} is only a few 16-bit ulps
# wide, so rounding each level loses most of it.  Measured f16 2.2e-3
# (64^3), 1.36e-2 / 5.8e-3 (crop); bf16 2.5e-2, 0.563 / 0.168.  Their crop
# bounds are regression bounds, about 1.15-1.25x the measured values (an
# all-zero field scores 1.0, a field off by one stored exponent 1.0 or
# more), stated separately for the field and the traces.
BOUND = {"f16": {"small": 4e-3, "crop": (1.6e-2, 7e-3)}, "bf16": {"small": 4e-2, "crop": (0.65, 0.2)},
         "f16uv": {"small": 2e-3, "crop": (6e-3, 6e-3)}, "bf16uv": {"small": 2e-2, "crop": (5e-2, 5e-2)}}
# the bounds proposed for reduced-precision storage, which the two-level
# forms miss on the crop
PROPOSED = {"f16": 5e-3, "bf16": 5e-2, "f16uv": 5e-3, "bf16uv": 5e-2}
LOWP = ["f16", "bf16", "f16uv", "bf16uv"]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(wave, p, dtype, variant=0, zchunk=0, src_scale=1.0, nt=None):
    nt = p.nt if nt is None else nt
    prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                           sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dtype)
    prop.configure(variant, zchunk)
    prop.record(nt)
    s = torch.tensor(np.asarray(p.s[:nt]) * src_scale, dtype=torch.float32, device="cuda")
    prop.run(nt, s)
    cur, prev, n = prop.fields()
    # raw stored bits (numpy has no bfloat16)
    raw = tuple(prop.padded(b).view(torch.int16 if b.element_size() == 2 else torch.int32)
                .cpu().numpy().copy() for b in (cur, prev))
    field = prop.export(0).cpu().numpy()
    prev_f = prop.export(1).cpu().numpy()
    prop.sync()
    tr = prop.traces.cpu().numpy()[:, :prop.nrec]
    prop.close()
    assert n == nt
    return field, prev_f, tr, raw


@pytest.fixture(scope="module")
def ragged():
    return inputs.random_problem(37, 21, 19, 40, seed=12, sponge_width=3, nrec=24)


@pytest.mark.parametrize("dtype", LOWP)
def test_kernels_bitwise_equal(wave_mod, ragged, dtype):
    ref = run(wave_mod, ragged, dtype, variant=1)
    for v in range(2, wave_mod.wave_variant_count()):
        for zc in (0, 1, 3, 19):
            print(f"case: {dtype} 37x21x19 variant {wave_mod.wave_variant_name(v)} zchunk {zc}",
                  flush=True)
            got = run(wave_mod, ragged, dtype, variant=v, zchunk=zc)
            assert np.array_equal(got[3][0], ref[3][0]), (v, zc)
            assert np.array_equal(got[3][1], ref[3][1]), (v, zc)
            assert np.array_equal(got[2], ref[2]), (v, zc)


@pytest.mark.parametrize("dtype", LOWP)
@pytest.mark.parametrize("j", [20, -30])
def test_power_of_two_equivariance(wave_mod, ragged, dtype, j):
    a = run(wave_mod, ragged, dtype)
    b = run(wave_mod, ragged, dtype, src_scale=2.0 ** j)
    assert np.array_equal(a[3][0], b[3][0]) and np.array_equal(a[3][1], b[3][1])
    tiny = np.finfo(np.float32).tiny
    for x, y in ((a[0], b[0]), (a[2], b[2])):
        xs = x * np.float32(2.0 ** j)
        normal = (np.abs(x) >= tiny) & (np.abs(y) >= tiny)
        assert np.array_equal(xs[normal], y[normal])
        assert np.all(np.abs(xs[~normal].astype(np.float64) - y[~normal]) <= tiny)
        assert normal.flat[np.argmax(np.abs(y))]  # the largest value is compared exactly


@pytest.mark.parametrize("dtype", LOWP)
def test_small_parity_accuracy(wave_mod, oracle_lib, dtype):
    p = inputs.small_parity()
    ref = oracle_lib.run(p.k64(), p.h, p.nt, s=p.s, src=p.src, rec=p.rec)
    f, pf, tr, _ = run(wave_mod, p, dtype)
    e_f, e_p = rel(f, ref[0]), rel(pf, ref[1])
    # (the 16 random receivers of this workload lie beyond the 100-step
    # wavefront and record only precursor amplitudes far below 16-bit
    # resolution; trace accuracy is checked on the crop)
    print(f"{dtype} 64^3 x 100: rel-L2 field {e_f:.3e} prev {e_p:.3e}")
    b = BOUND[dtype]["small"]
    assert e_f <= b and e_p <= b


@pytest.fixture(scope="module")
def crop():
    return inputs.crop_shot()


@pytest.fixture(scope="module")
def crop_ref(oracle_lib, crop):
    p = crop
    return oracle_lib.run(p.k64(), p.h, p.nt, s=p.s, src=p.src, rec=p.rec,
                          sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)


@pytest.mark.parametrize("dtype", ["f32"] + LOWP)
def test_crop_accuracy(wave_mod, crop, crop_ref, dtype):
    f, _, tr, _ = run(wave_mod, crop, dtype)
    e_f, e_t = rel(f, crop_ref[0]), rel(tr, crop_ref[2])
    print(f"{dtype} 128^3 crop x 500: rel-L2 field {e_f:.3e} traces {e_t:.3e}")
    b_f, b_t = (1e-5, 1e-5) if dtype == "f32" else BOUND[dtype]["crop"]
    assert e_f <= b_f and e_t <= b_t
    if dtype.endswith("uv"):
        assert max(e_f, e_t) <= PROPOSED[dtype]


def test_f32_export_is_a_copy(wave_mod, ragged):
    p = ragged
    prop = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src)
    prop.run(p.nt, torch.tensor(p.s, dtype=torch.float32, device="cuda"))
    cur, prev, _ = prop.fields()
    assert torch.equal(prop.export(0), prop.interior(cur))
    assert torch.equal(prop.export(1), prop.interior(prev))
    prop.close()


@pytest.mark.parametrize("dtype", LOWP)
def test_stored_magnitude_stays_below_two_to_fourteen(wave_mod, ragged, dtype):
    # the chosen exponent keeps every stored value below 2^14 (FP16 max 65504)
    p = ragged
    prop = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, dtype=dtype)
    s = torch.tensor(p.s * 1e6, dtype=torch.float32, device="cuda")
    for j in range(p.nt):
        prop.run(1, s[j:])
        cur, _, _ = prop.fields()
        m = prop.interior(cur).float().abs().max().item()
        assert np.isfinite(m) and m < 2.0 ** 14
    prop.close()


def emulation_check(wave, oracle_lib, p, dtype):
    # the GPU's stored 16-bit field, its level exponent and its traces against
    # the CPU emulation of the same scheme (oracle/oracle16.c: FP32 arithmetic
    # in the documented order, its own codecs and exponent rule), both run
    # for the same steps from zero fields; in the u-and-change forms d^n
    # enters every later level, so equal levels pin it up to the last step
    s32 = p.s.astype(np.float32)
    print(f"case: {dtype} {p.nx}x{p.ny}x{p.nz} x {p.nt} steps against the emulation", flush=True)
    prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                           sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dtype)
    prop.record(p.nt)
    prop.run(p.nt, torch.tensor(s32, device="cuda"))
    cur, _, n = prop.fields()
    bits = prop.interior(cur).view(torch.int16).cpu().numpy().view(np.uint16).copy()
    dec = prop.export(0).cpu().numpy()
    prop.sync()
    tr = prop.traces.cpu().numpy()[:, :prop.nrec]
    prop.close()
    assert n == p.nt
    u, _, exps, rtr = oracle_lib.run16(p.k32(), p.h, p.nt, dtype, s=s32, src=p.src, rec=p.rec,
                                       sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    diff = int(np.count_nonzero(bits != u))
    # the GPU's exponent of the last level: decoded export over stored value
    _, dec16 = oracle_lib.codec16("bf16" if dtype.startswith("bf16") else "f16")
    i = np.unravel_index(np.argmax(np.abs(dec)), dec.shape)
    e_gpu = int(np.round(np.log2(abs(float(dec[i])) / abs(dec16(int(bits[i]))))))
    print(f"{dtype}: {diff} of {bits.size} stored values differ; exponent GPU {e_gpu}, emulation {exps[-1]}; "
          f"traces equal: {np.array_equal(tr, rtr)}")
    assert diff == 0
    assert e_gpu == exps[-1]
    assert np.array_equal(tr, rtr)


@pytest.mark.parametrize("dtype", LOWP)
def test_bitwise_equal_to_cpu_emulation(wave_mod, oracle_lib, ragged, dtype):
    emulation_check(wave_mod, oracle_lib, ragged, dtype)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype", LOWP)
def test_crop_bitwise_equal_to_cpu_emulation(wave_mod, oracle_lib, crop, dtype):
    # 128^3, 500 steps, sponge 20 cells: several tiles and chunks, and the
    # exponent rule over hundreds of levels (the emulation takes ~10-20 s)
    emulation_check(wave_mod, oracle_lib, crop, dtype)
