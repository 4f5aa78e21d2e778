"""FP64 CPU oracle for the 25-point leapfrog wave propagator (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
CPU-baseline leg of the benchmark use this package; the product path never
imports it.  It shares no code with the HIP library: ``oracle.c`` restates the
paper's method (Section III: Eq. 1, Eq. 2, the 25-point Laplacian and
Algorithm 1; Section IV-B ghost cells; Section IV-C centre folding; Section
IV-D source injection) as plain loops in double precision.

All arrays are dense interior arrays ``[nz][ny][nx]`` (x fastest) unless a
function says it takes a padded array ``[nz+8][ny+8][nx+8]``.

Parity status per function (what pins it lives in ``tests/test_oracle_*``):
  coefficients     pinned (exact rationals, moment conditions, degree-10 residual)
  laplacian        pinned (polynomial exactness, degree-10 error, convergence,
                   Kronecker-sum brute force)
  run              pinned (impulse response, plane-wave dispersion, energy,
                   reciprocity, brute force, restart equivalence; the sponge
                   damping both time levels: on one cell u^{n+1} = G^n w^{n+1},
                   w the undamped recurrence)
  sponge_profile   parity unpinned beyond W = 0 reduction and its own
                   definition (the sponge is a chosen published method, not
                   something the paper fixes)
  step_points      pinned against ``run`` (same update, pointwise)
  adjoint          pinned (central finite differences of the misfit computed
                   with ``run``, single cells inside and outside the sponge
                   and a random direction; dot-product identity against
                   ``tangent`` to FP64 rounding)
  tangent          pinned (central finite differences of the traces computed
                   with ``run``, converging as eps^2)
  run16            the 16-bit storage forms (an extension of the paper's FP32
                   scheme) emulated in FP32: codecs pinned against numpy's
                   binary16 and an independent nearest-even bfloat16
                   rounding; each step against the FP64 update of its own
                   decoded inputs; exact power-of-two equivariance
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "oracle.c")

BC_ZERO = 0
BC_PERIODIC = 1

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (see oracle/Makefile: gcc, FP64,
    no fast-math, no FMA contraction)."""
    cmd = ["make", "-s", "-C", _HERE] + (["-B"] if force else [])
    subprocess.run(cmd, check=True)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    ci, cd = ctypes.c_int, ctypes.c_double
    lib.oracle_coefficients.argtypes = [dp]
    lib.oracle_coefficients.restype = None
    lib.oracle_sponge_profile.argtypes = [ci, ci, cd, dp]
    lib.oracle_sponge_profile.restype = None
    lib.oracle_laplacian.argtypes = [ci, ci, ci, cd, cd, cd, dp, dp, ci]
    lib.oracle_laplacian.restype = ci
    lib.oracle_run.argtypes = [ci, ci, ci, cd, cd, cd, ci, ci, cd, dp, ci, dp, ci, ci, ci,
                               ci, ip, dp, dp, dp, ci]
    lib.oracle_run.restype = ci
    lib.oracle_step_points.argtypes = [ci, ci, ci, cd, cd, cd, ci, cd, fp, fp, fp, ci, ci,
                                       ci, ci, cd, ci, ip, dp]
    lib.oracle_step_points.restype = ci
    lib.oracle_adjoint.argtypes = [ci, ci, ci, cd, cd, cd, ci, cd, dp, ci, dp, ci, ci, ci, ci, ip,
                                   dp, dp, ci]
    lib.oracle_adjoint.restype = ci
    lib.oracle_tangent.argtypes = [ci, ci, ci, cd, cd, cd, ci, cd, dp, dp, ci, dp, ci, ci, ci, ci, ip,
                                   dp, ci]
    lib.oracle_tangent.restype = ci
    u16p = ctypes.POINTER(ctypes.c_uint16)
    lib.oracle16_run.argtypes = [ci, ci, ci, cd, cd, cd, ci, cd, ci, fp, ci, fp, ci, ci, ci, ci, ip, u16p, u16p,
                                 ip, fp]
    lib.oracle16_run.restype = ci
    lib.oracle16_f16_encode.argtypes = [ctypes.c_float]
    lib.oracle16_f16_encode.restype = ctypes.c_uint16
    lib.oracle16_f16_decode.argtypes = [ctypes.c_uint16]
    lib.oracle16_f16_decode.restype = ctypes.c_float
    lib.oracle16_bf16_encode.argtypes = [ctypes.c_float]
    lib.oracle16_bf16_encode.restype = ctypes.c_uint16
    lib.oracle16_bf16_decode.argtypes = [ctypes.c_uint16]
    lib.oracle16_bf16_decode.restype = ctypes.c_float
    _lib = lib
    return lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def coefficients() -> np.ndarray:
    """c_0..c_4 of the 8th-order second derivative (closed form, FP64)."""
    c = np.zeros(5, dtype=np.float64)
    _load().oracle_coefficients(_dptr(c))
    return c


def sponge_profile(n: int, width: int, alpha: float) -> np.ndarray:
    g = np.zeros(n, dtype=np.float64)
    _load().oracle_sponge_profile(int(n), int(width), float(alpha), _dptr(g))
    return g


def laplacian(a_pad: np.ndarray, h, nthreads: int | None = None) -> np.ndarray:
    """25-point Laplacian of a padded array [nz+8][ny+8][nx+8] (ghost values as
    given); returns the interior [nz][ny][nx].  ``h`` = (dx, dy, dz)."""
    a_pad = np.ascontiguousarray(a_pad, dtype=np.float64)
    nz, ny, nx = (d - 8 for d in a_pad.shape)
    out = np.zeros((nz, ny, nx), dtype=np.float64)
    dx, dy, dz = h
    rc = _load().oracle_laplacian(nx, ny, nz, dx, dy, dz, _dptr(a_pad), _dptr(out),
                                  nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_laplacian rejected its arguments (rc={rc})")
    return out


def run(k: np.ndarray, h, nt: int, *, s=None, src=(0, 0, 0), rec=None, a_cur=None,
        a_prev=None, sponge_width: int = 0, sponge_alpha: float = 0.0, bc: int = BC_ZERO,
        nthreads: int | None = None):
    """Run ``nt`` steps.  Returns (a_cur, a_prev, traces): u^{n0+nt},
    u^{n0+nt-1} and traces [nt][nrec] (row j = field after step j)."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    nz, ny, nx = k.shape
    dx, dy, dz = h
    a_cur = np.zeros_like(k) if a_cur is None else np.array(a_cur, dtype=np.float64, copy=True)
    a_prev = np.zeros_like(k) if a_prev is None else np.array(a_prev, dtype=np.float64, copy=True)
    assert a_cur.shape == k.shape and a_prev.shape == k.shape
    rec = np.zeros((0, 3), dtype=np.int32) if rec is None else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3)
    nrec = rec.shape[0]
    traces = np.zeros((max(nt, 0), nrec), dtype=np.float64)
    if s is not None:
        s = np.ascontiguousarray(s, dtype=np.float64)
        assert s.shape[0] >= nt
        sp = _dptr(s)
    else:
        sp = None
    rc = _load().oracle_run(nx, ny, nz, dx, dy, dz, int(bc), int(sponge_width), float(sponge_alpha),
                            _dptr(k), int(nt), sp, int(src[0]), int(src[1]), int(src[2]), nrec,
                            _iptr(rec), _dptr(a_cur), _dptr(a_prev), _dptr(traces),
                            nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_run rejected its arguments (rc={rc})")
    return a_cur, a_prev, traces


def run_segments(k: np.ndarray, h, nt: int, segment: int, *, s=None, progress=None, **kw):
    """``run`` over ``nt`` steps as consecutive calls of at most ``segment``
    steps, each restarting from the levels the previous one returned (the
    restart is bitwise, see the restart pin), so that a long run can report
    progress between segments.  ``progress(done, nt, seconds)`` is called
    after each segment.  Returns (a_cur, a_prev, traces, seconds spent in
    ``run``)."""
    import time

    k = np.ascontiguousarray(k, dtype=np.float64)
    a_cur = a_prev = None
    rows = []
    done, sec = 0, 0.0
    while done < nt:
        n = min(segment, nt - done)
        t0 = time.perf_counter()
        a_cur, a_prev, tr = run(k, h, n, s=None if s is None else np.asarray(s)[done:], a_cur=a_cur,
                                a_prev=a_prev, **kw)
        sec += time.perf_counter() - t0
        rows.append(tr)
        done += n
        if progress is not None:
            progress(done, nt, sec)
    if a_cur is None:
        a_cur, a_prev, tr = run(k, h, 0, s=s, **kw)
        rows.append(tr)
    return a_cur, a_prev, np.concatenate(rows, axis=0), sec


FORMS16 = {"f16": 1, "bf16": 2, "f16uv": 3, "bf16uv": 4}


def codec16(form: str):
    """(encode, decode) of one 16-bit value for "f16" or "bf16" (scalar
    functions of the emulation, for its own pins)."""
    lib = _load()
    if form == "f16":
        return lib.oracle16_f16_encode, lib.oracle16_f16_decode
    return lib.oracle16_bf16_encode, lib.oracle16_bf16_decode


def run16(k32, h, nt: int, form: str, *, s=None, src=None, rec=None, sponge_width: int = 0,
          sponge_alpha: float = 0.0):
    """The 16-bit storage forms emulated in FP32 on the CPU (oracle16.c):
    ``nt`` steps from zero fields with FP32 k ``k32`` [nz][ny][nx] and FP32
    source values ``s``.  Returns (stored u^nt bits [nz][ny][nx] uint16,
    stored d^nt bits or None, exponents [nt] of u^1..u^nt, traces [nt][nrec]
    FP32)."""
    k32 = np.ascontiguousarray(k32, dtype=np.float32)
    nz, ny, nx = k32.shape
    dx, dy, dz = h
    f = FORMS16[form]
    rec = np.zeros((0, 3), dtype=np.int32) if rec is None else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3)
    nrec = rec.shape[0]
    u = np.zeros((nz, ny, nx), dtype=np.uint16)
    d = np.zeros((nz, ny, nx), dtype=np.uint16) if f >= 3 else None
    exps = np.zeros(max(nt, 0), dtype=np.int32)
    traces = np.zeros((max(nt, 0), nrec), dtype=np.float32)
    sp = None
    if s is not None:
        s = np.ascontiguousarray(s, dtype=np.float32)
        assert s.shape[0] >= nt
        sp = _fptr(s)
    sz, sy, sx = src if src is not None else (-1, -1, -1)
    u16 = ctypes.POINTER(ctypes.c_uint16)
    rc = _load().oracle16_run(nx, ny, nz, dx, dy, dz, int(sponge_width), float(sponge_alpha), f, _fptr(k32),
                              int(nt), sp, int(sz), int(sy), int(sx), nrec, _iptr(rec),
                              u.ctypes.data_as(u16), d.ctypes.data_as(u16) if d is not None else None,
                              _iptr(exps), _fptr(traces))
    if rc != 0:
        raise ValueError(f"oracle16_run rejected its arguments (rc={rc})")
    return u, d, exps, traces


def step_points(k32, u_cur32, u_prev32, h, pts, *, sponge_width=0, sponge_alpha=0.0,
                src=None, src_value=0.0) -> np.ndarray:
    """One update at the listed points [npts][3] (z, y, x), in FP64 from FP32
    copies of k, u^n and u^{n-1}."""
    k32 = np.ascontiguousarray(k32, dtype=np.float32)
    u_cur32 = np.ascontiguousarray(u_cur32, dtype=np.float32)
    u_prev32 = np.ascontiguousarray(u_prev32, dtype=np.float32)
    nz, ny, nx = k32.shape
    pts = np.ascontiguousarray(pts, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    dx, dy, dz = h
    has_src = src is not None
    sz, sy, sx = src if has_src else (0, 0, 0)
    rc = _load().oracle_step_points(nx, ny, nz, dx, dy, dz, int(sponge_width), float(sponge_alpha),
                                    _fptr(k32), _fptr(u_cur32), _fptr(u_prev32), int(has_src),
                                    int(sz), int(sy), int(sx), float(src_value), pts.shape[0],
                                    _iptr(pts), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle_step_points rejected its arguments (rc={rc})")
    return out


def adjoint(k: np.ndarray, h, nt: int, trace_grad, *, s=None, src=(0, 0, 0), rec=None,
            sponge_width: int = 0, sponge_alpha: float = 0.0, nthreads: int | None = None):
    """Gradient with respect to k (dense [nz][ny][nx], FP64) of a loss whose
    derivative with respect to the traces [nt][nrec] is ``trace_grad``."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    nz, ny, nx = k.shape
    dx, dy, dz = h
    rec = np.zeros((0, 3), dtype=np.int32) if rec is None else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3)
    tg = np.ascontiguousarray(trace_grad, dtype=np.float64).reshape(nt, rec.shape[0])
    grad = np.zeros_like(k)
    sp = None
    if s is not None:
        s = np.ascontiguousarray(s, dtype=np.float64)
        sp = _dptr(s)
    rc = _load().oracle_adjoint(nx, ny, nz, dx, dy, dz, int(sponge_width), float(sponge_alpha),
                                _dptr(k), int(nt), sp, int(src[0]), int(src[1]), int(src[2]),
                                rec.shape[0], _iptr(rec), _dptr(tg), _dptr(grad),
                                nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_adjoint rejected its arguments (rc={rc})")
    return grad


def tangent(k: np.ndarray, dk: np.ndarray, h, nt: int, *, s=None, src=(0, 0, 0), rec=None,
            sponge_width: int = 0, sponge_alpha: float = 0.0, nthreads: int | None = None):
    """Derivative of the traces [nt][nrec] with respect to k along ``dk``
    (tangent-linear run from zero initial levels; source values fixed)."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    dk = np.ascontiguousarray(dk, dtype=np.float64)
    if dk.shape != k.shape:
        raise ValueError("dk must have the shape of k")
    nz, ny, nx = k.shape
    dx, dy, dz = h
    rec = np.zeros((0, 3), dtype=np.int32) if rec is None else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((nt, rec.shape[0]), dtype=np.float64)
    sp = None
    if s is not None:
        s = np.ascontiguousarray(s, dtype=np.float64)
        sp = _dptr(s)
    rc = _load().oracle_tangent(nx, ny, nz, dx, dy, dz, int(sponge_width), float(sponge_alpha),
                                _dptr(k), _dptr(dk), int(nt), sp, int(src[0]), int(src[1]), int(src[2]),
                                rec.shape[0], _iptr(rec), _dptr(out), nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_tangent rejected its arguments (rc={rc})")
    return out
