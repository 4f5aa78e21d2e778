"""C ABI checks that need no GPU: the library loads, exports every function
include/wave.h declares, computes layouts, and rejects bad arguments before
touching the device."""
import ctypes
import re

import pytest


@pytest.fixture(scope="module")
def w(wave_mod):
    return wave_mod


def _declared_functions(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(wave_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(w):
    names = _declared_functions(w.HEADER)
    assert len(names) >= 15, names
    lib = ctypes.CDLL(w.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_every_probe_symbol_is_exported(w):
    # include/wave_probe.h declares the measurement probes of libwave_probe.so
    import os

    header = os.path.join(os.path.dirname(w.HEADER), "wave_probe.h")
    text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    names = sorted(set(re.findall(r"^\s*int\s+(probe_[a-z_0-9]+)\s*\(", text, flags=re.M)))
    assert {"probe_copy", "probe_read3_write1", "probe_adjoint_mix", "probe_sync", "probe_empty"} <= set(names)
    from paper_2204_03775_amd import probe

    lib = probe._load()
    for n in names:
        assert hasattr(lib, n), n
    assert lib.probe_sync(None, 256, 10, 0, 1.0, None) == -1  # rejected before any launch
    assert lib.probe_empty(0, None) == -1


def test_single_hip_runtime_in_process(w):
    maps = open("/proc/self/maps").read()
    paths = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(paths) == 1, paths


def test_layout_arithmetic(w):
    L = w.wave_layout(512, 512, 512)
    assert L.x_offset == 32
    assert L.pitch_x % 32 == 0 and L.pitch_x >= 32 + 512 + 4
    assert (L.rows, L.planes) == (520, 520)
    assert L.plane == L.pitch_x * L.rows
    assert L.elems == L.plane * L.planes and L.bytes == 4 * L.elems
    for nx in (1, 3, 4, 5, 63, 64, 65, 127):
        L = w.wave_layout(nx, 7, 9)
        nxq = (nx + 3) // 4
        # the float4 right of the last partial one (ghost reads) must fit in the row
        assert L.pitch_x >= L.x_offset + 4 * nxq + 4
        assert L.pitch_x % 32 == 0


@pytest.mark.parametrize("dims", [(0, 4, 4), (4, -1, 4), (4, 4, 0)])
def test_layout_rejects_bad_sizes(w, dims):
    with pytest.raises(w.WaveError) as e:
        w.wave_layout(*dims)
    assert e.value.code == w.WAVE_EINVAL


def test_layout_rejects_unknown_dtype(w):
    with pytest.raises(w.WaveError):
        w.wave_layout(8, 8, 8, 7)


def _params(w, **kw):
    p = dict(nx=8, ny=8, nz=8, dx=10.0, dy=10.0, dz=10.0, sponge_width=0, sponge_alpha=0.0,
             dtype=0)
    p.update(kw)
    return w.wave_params_t(**p)


# A fake, 256-byte aligned "device" address: wave_init must reject the call
# while validating, before it could dereference anything.
FAKE = 0x7f0000000000


@pytest.mark.parametrize("kw", [dict(nx=0), dict(dx=0.0), dict(dy=-1.0), dict(dz=float("nan")),
                                dict(sponge_width=-1), dict(sponge_alpha=-0.1), dict(dtype=5)])
def test_init_rejects_bad_params(w, kw):
    with pytest.raises(w.WaveError) as e:
        w.wave_init(_params(w, **kw), FAKE, FAKE + 4096, FAKE + 8192)
    assert e.value.code == w.WAVE_EINVAL


def test_init_rejects_bad_pointers_and_points(w):
    p = _params(w)
    cases = [
        (0, FAKE, FAKE + 4096, None, None),          # NULL k
        (FAKE, FAKE + 4096, FAKE + 4096, None, None),  # cur == prev
        (FAKE + 2, FAKE + 4096, FAKE + 8192, None, None),  # misaligned
        (FAKE, FAKE + 4096, FAKE + 8192, (8, 0, 0), None),  # source outside
        (FAKE, FAKE + 4096, FAKE + 8192, None, [[0, 0, 0], [0, -1, 0]]),  # receiver outside
    ]
    for k, c, pr, src, rec in cases:
        with pytest.raises(w.WaveError) as e:
            w.wave_init(p, k, c, pr, src, rec)
        assert e.value.code == w.WAVE_EINVAL


def test_null_context_calls(w):
    lib = w.lib()
    assert lib.wave_step(None, 0.0) == w.WAVE_EINVAL
    assert lib.wave_run(None, 1, None) == w.WAVE_EINVAL
    assert lib.wave_sync(None) == w.WAVE_EINVAL
    assert lib.wave_destroy(None) == w.WAVE_OK


def test_strerror_and_variants(w):
    for code in (0, -1, -2, -3, -4, -5):
        assert w.wave_strerror(code)
    assert w.wave_strerror(-99) == "unknown error"
    names = w.variants()
    assert names["auto"] == 0 and names["naive"] == 1
    assert len(names) == w.wave_variant_count() >= 3
    assert w.wave_variant_name(w.wave_variant_count()) is None


def test_gradient_calls_reject_null_context(w):
    lib = w.lib()
    assert lib.wave_forward_checkpointed(None, 10, None, 0) == w.WAVE_EINVAL
    assert lib.wave_adjoint(None, None, None, 0) == w.WAVE_EINVAL
    assert lib.wave_grad_info(None, None, None, None, None) == w.WAVE_EINVAL


def test_misfit_rejects_bad_arguments(w):
    lib = w.lib()
    dummy = ctypes.c_void_p(16)  # never dereferenced: rejected before any launch
    assert lib.wave_misfit(dummy, dummy, -1, None, dummy, None) == w.WAVE_EINVAL
    assert lib.wave_misfit(dummy, dummy, 4, None, None, None) == w.WAVE_EINVAL
    assert lib.wave_misfit(None, dummy, 4, None, dummy, None) == w.WAVE_EINVAL


def test_check_rejects_null_context(w):
    assert w.lib().wave_check(None, None, None) == w.WAVE_EINVAL


def test_batch_calls_reject_null_handles(w):
    lib = w.lib()
    out = ctypes.c_void_p(0)
    assert lib.wave_batch_create(None, None, 1, None, 0) == w.WAVE_EINVAL
    assert lib.wave_batch_create(ctypes.byref(out), None, 1, None, 0) == w.WAVE_EINVAL
    assert out.value is None
    assert lib.wave_batch_run(None, 1, None) == w.WAVE_EINVAL
    assert lib.wave_batch_set_schedule(None, 1, 2) == w.WAVE_EINVAL
    assert lib.wave_batch_set_wait_limit(None, 1) == w.WAVE_EINVAL
    assert lib.wave_batch_info(None, None, None, None) == w.WAVE_EINVAL
    assert lib.wave_batch_sync(None) == w.WAVE_EINVAL
    assert lib.wave_batch_destroy(None) == w.WAVE_OK
    assert lib.wave_batch_last_error(None) == b""
