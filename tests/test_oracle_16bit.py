"""Pins of the CPU emulation of the 16-bit storage forms (oracle/oracle16.c).

Storing fields in 16 bits is this project's extension of the paper's FP32
scheme (its Eq. 2 update is unchanged); the emulation carries the scheme
out in FP32 on the CPU so that GPU runs can be compared with it bit for
bit.  It is pinned here against things outside itself:
  - the binary16 codec against numpy's float16 conversions (IEEE binary16,
    round to nearest even, subnormals) on every bit pattern and on random,
    tie and boundary values;
  - the bfloat16 codec against the nearest-even rounding computed
    independently in FP64 from the two neighbouring bfloat16 values;
  - every emulated step against the FP64 update of its own decoded inputs
    (the FP64 oracle's pointwise step), within the rounding the step's FP32
    arithmetic and 16-bit output allow;
  - the headroom the level exponents leave: every stored maximum within
    the range the exponent rule implies for this wave;
  - power-of-two equivariance of the level exponents: scaling the source by
    2^j leaves every stored bit unchanged and moves every exponent by j."""
import numpy as np
import pytest

from paper_2204_03775_amd import inputs

FORMS = ["f16", "bf16", "f16uv", "bf16uv"]


def test_f16_codec_matches_numpy(oracle_lib):
    enc, dec = oracle_lib.codec16("f16")
    bits = np.arange(65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float32)
    for b in range(0, 65536, 7):  # every 7th pattern, NaNs excluded
        if not np.isnan(ref[b]):
            assert dec(int(b)) == ref[b], b
    rng = np.random.default_rng(16)
    vals = [np.float32(v) for v in rng.standard_normal(4000) * np.exp2(rng.integers(-30, 17, 4000))]
    # exact ties: half-way between neighbouring binary16 values (normal and subnormal)
    for h in (np.float16(1.0), np.float16(3.0e-6), np.float16(0.000123), np.float16(1000.5), np.float16(-7.25)):
        nxt = np.nextafter(h, np.float16(np.inf), dtype=np.float16)
        vals.append(np.float32((np.float64(h) + np.float64(nxt)) / 2))
    vals += [np.float32(v) for v in (65504.0, 65519.99, 65520.0, -65520.0, 1e-9, 5.96e-8, 2.98e-8, 0.0, -0.0)]
    with np.errstate(over="ignore"):  # numpy warns when it rounds to infinity
        for v in vals:
            assert enc(float(v)) == int(np.float16(v).view(np.uint16)), v


def _bf16_nearest_even(x: np.float32) -> int:
    u = int(np.float32(x).view(np.uint32))
    lo = u & 0xFFFF0000
    hi = (lo + 0x10000) & 0xFFFFFFFF
    a = float(np.uint32(lo).view(np.float32))
    b = float(np.uint32(hi).view(np.float32))
    xd = float(x)
    da, db = abs(xd - a), abs(b - xd)
    if da < db or (da == db and ((lo >> 16) & 1) == 0):
        return lo >> 16
    return hi >> 16


def test_bf16_codec_is_nearest_even(oracle_lib):
    enc, dec = oracle_lib.codec16("bf16")
    for b in range(0, 65536, 5):
        v = np.uint32(b << 16).view(np.float32)
        if not np.isnan(v):
            assert dec(b) == v, b
    rng = np.random.default_rng(17)
    vals = list((rng.standard_normal(4000) * np.exp2(rng.integers(-120, 120, 4000))).astype(np.float32))
    for base in (1.0, 3.0, -5.5, 1e-30):
        u = int(np.float32(base).view(np.uint32)) & 0xFFFF0000
        vals.append(np.uint32(u | 0x8000).view(np.float32))          # tie, even below
        vals.append(np.uint32((u + 0x10000) | 0x8000).view(np.float32))  # tie, odd below
    for v in vals:
        assert enc(float(v)) == _bf16_nearest_even(np.float32(v)), v


def _decode(oracle_lib, form, bits, e):
    _, dec = oracle_lib.codec16("bf16" if form.startswith("bf16") else "f16")
    lut = np.array([dec(i) for i in range(65536)], dtype=np.float64)
    return lut[bits.astype(np.int64)] * 2.0 ** e


@pytest.fixture(scope="module")
def prob():
    return inputs.random_problem(19, 15, 11, 24, seed=23, sponge_width=3, sponge_alpha=0.08, nrec=6)


@pytest.mark.parametrize("form", FORMS)
def test_each_step_is_the_fp64_update_of_its_inputs(oracle_lib, prob, form):
    # the last step, made from the emulation's own stored levels: u^{n} and
    # u^{n-1} (two levels) or d^{n} = u^{n} - u^{n-1} (u and change), and the
    # stored k, all decoded exactly; the FP64 update of those values is what
    # the FP32 arithmetic approximates before the result is rounded to 16
    # bits (half an ulp of the output format, eps/2 relative)
    p = prob
    s32 = p.s.astype(np.float32)
    kw = dict(s=s32, src=p.src, rec=p.rec, sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    nt = p.nt
    u1, d1, e1, _ = oracle_lib.run16(p.k32(), p.h, nt - 1, form, **kw)
    u0, _, e0, _ = oracle_lib.run16(p.k32(), p.h, nt - 2, form, **kw)
    u2, _, e2, tr = oracle_lib.run16(p.k32(), p.h, nt, form, **kw)
    cur = _decode(oracle_lib, form, u1, e1[-1])
    if form.endswith("uv"):
        prev = cur - _decode(oracle_lib, form, d1, e1[-1] + 1)
        # u^{n-1} rebuilt from u^n and the stored change is the level stored
        # a step earlier, up to the rounding of the two stored values
        ref_prev = _decode(oracle_lib, form, u0, e0[-1])
        eps_f = 2.0 ** (-11 if form.startswith("f16") else -8)
        assert np.abs(prev - ref_prev).max() <= 2 * eps_f * np.abs(ref_prev).max()
    else:
        prev = _decode(oracle_lib, form, u0, e0[-1])
    # k as the emulation stores it: one exponent ek with max k below 2^14 * 2^ek
    kmax = float(p.k32().max())
    ek = int(np.frexp(kmax)[1]) - 14
    kbits = np.array([oracle_lib.codec16("bf16" if form.startswith("bf16") else "f16")[0](float(v))
                      for v in (p.k32() * np.float32(2.0 ** -ek)).ravel()], dtype=np.uint16).reshape(p.shape)
    kdec = _decode(oracle_lib, form, kbits, ek)
    nz, ny, nx = p.shape
    pts = np.argwhere(np.ones(p.shape, dtype=bool)).astype(np.int32)
    ref = oracle_lib.step_points(kdec.astype(np.float32), cur.astype(np.float32), prev.astype(np.float32), p.h, pts,
                                 sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, src=p.src,
                                 src_value=float(s32[nt - 1]))
    # the decoded inputs are exact FP32 values (16-bit values times powers of two)
    assert np.array_equal(cur.astype(np.float32).astype(np.float64), cur)
    got = _decode(oracle_lib, form, u2, e2[-1]).ravel()
    eps = 2.0 ** (-11 if form.startswith("f16") else -8)
    M = max(np.abs(cur).max(), np.abs(prev).max())
    err = np.abs(got - ref)
    print(f"{form}: max |diff| {err.max():.3e} = {err.max() / (eps * M):.3f} eps M")
    assert err.max() <= 8 * eps * M
    # the largest stored magnitude of the last level: the rule puts 8 M in
    # [2^13, 2^14) stored units, and this wave's maximum changed little over
    # the last steps, so it lies in [2^10, 2^11) (measured 1394..1400)
    raw = np.abs(_decode(oracle_lib, form, u2, 0))
    assert 2.0 ** 10 <= raw.max() < 2.0 ** 11
    # the last trace row is the decoded u^{nt} at the receivers
    rz, ry, rx = np.asarray(p.rec).T
    assert np.array_equal(tr[-1], got.reshape(p.shape)[rz, ry, rx].astype(np.float32))


@pytest.mark.parametrize("form", FORMS)
def test_level_exponents_leave_the_stated_headroom(oracle_lib, prob, form):
    # the exponent of each level puts 8 max(M_n, M_{n-1}) + |s_n| in
    # [2^13, 2^14) stored units; the levels of this wave change their maximum
    # by less than a factor 2 from step to step, so every stored maximum from
    # the second level on lies in [2^10, 2^13) (measured 1270..5056): an
    # exponent one off either way moves them out
    p = prob
    kw = dict(s=p.s.astype(np.float32), src=p.src, rec=p.rec, sponge_width=p.sponge_width,
              sponge_alpha=p.sponge_alpha)
    for n in range(2, p.nt + 1):
        u, _, _, _ = oracle_lib.run16(p.k32(), p.h, n, form, **kw)
        raw = np.abs(_decode(oracle_lib, form, u, 0)).max()
        assert 2.0 ** 10 <= raw < 2.0 ** 13, (n, raw)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("j", [9, -13])
def test_power_of_two_equivariance(oracle_lib, prob, form, j):
    p = prob
    kw = dict(src=p.src, rec=p.rec, sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    s32 = p.s.astype(np.float32)
    a = oracle_lib.run16(p.k32(), p.h, p.nt, form, s=s32, **kw)
    b = oracle_lib.run16(p.k32(), p.h, p.nt, form, s=s32 * np.float32(2.0 ** j), **kw)
    assert np.array_equal(a[0], b[0])
    if a[1] is not None:
        assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2] + j, b[2])
    assert np.array_equal(a[3] * np.float32(2.0 ** j), b[3])
