// libwave.so: time stepping of the 3-D acoustic wave equation with the
// 25-point, 8th-order Laplacian inside a leapfrog update (paper Section III:
// Eq. 2, the Laplacian and Algorithm 1), written for MI355X (gfx950, CDNA4,
// wave64).  The C ABI is declared in include/wave.h.
//
// Kernel design.  The paper maps X and Y onto its processor grid and keeps
// the whole Z column in each processor's memory (Section IV-B); a GPU has a
// memory hierarchy instead, so the mapping here is the usual 2.5-D one:
//   - a work-group owns an x-y tile and a range of z planes and marches
//     through them;
//   - each thread owns 4 consecutive x cells in RY rows and keeps its z
//     column z-4 .. z+4 in a register queue (the GPU counterpart of the
//     paper's z update from local memory, Section IV-C);
//   - the centre plane of the tile, with a 4-cell halo in x and y, is
//     staged in LDS (double buffered: one barrier per plane) and the x and
//     y taps are read from there;
//   - the next plane, the halo and u^{n-1}, k are prefetched one plane
//     ahead so that HBM reads overlap the arithmetic;
//   - sponge, source injection and receiver sampling are fused: the
//     update, the source add and a per-work-group receiver epilogue happen
//     in the same launch.
// The step is bound by HBM bandwidth (about 3 flop per byte against a ridge
// near 20 for FP32 vector math), so nothing here uses the matrix cores.
//
// Laplacian form.  With FP32 fields the Laplacian is evaluated as
//   sum_a sum_m (c_m / h_a^2) (u(+m e_a) + u(-m e_a) - 2 u),
// which equals the paper's form because c_0 = -2 sum c_m, and which maps a
// constant to exactly zero whatever the rounding of the FP32 weights.  The
// classic form c_0 u + sum c_m (...) with FP32-rounded weights does not,
// and the small spurious mass term it leaves shifts the phase by about
// 2e-5 over five wavelengths at 17 cells per wavelength.  16-bit storage
// rounds each stored value far more coarsely than that, so those kernels
// keep the classic form and its 12 fewer operations per cell.
//
// Storage.  Fields are FP32, or FP16 / BF16 with FP32 arithmetic: a 16-bit
// field holds x * 2^-e for one exponent e per time level, chosen on the
// device when the level is written so that the largest value stays below
// 2^14 (see step_scales).  Decoding multiplies by 2^e, which is exact.

#pragma once

#include <type_traits>
#include <utility>

#include "wave_dev.h"

namespace wavek {

__device__ __forceinline__ float src_value(const StepArgs &a)
{
    return a.src_ptr ? a.src_ptr[0] : a.src_val;
}

// x * g rounded on its own.  The adjoint scales every loaded value by the
// sponge factor; if that product were contracted into the first sum that
// uses it (an FMA), the value would enter that sum unrounded and the other
// operand rounded, so the result would depend on which of u[z+m], u[z-m]
// was loaded last, i.e. on the direction of the z-march.
__device__ __forceinline__ float mul_rounded(float x, float g)
{
#pragma clang fp contract(off)
    return x * g;
}

// Work-groups are handed to the 8 XCDs round-robin by block index (the
// starting XCD follows on from the previous launch, so blocks with equal
// b % 8 share an XCD, not necessarily XCD b % 8); map block b to logical
// work-group (b % 8) * (G / 8) + b / 8 so that each XCD gets a contiguous
// run of neighbouring tiles whose halos share its L2.
__device__ __forceinline__ int logical_wg()
{
    const int b = blockIdx.x;
    const int per = gridDim.x >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// storage formats

template <int KIND>
struct Store;
template <>
struct Store<WAVE_F32> {
    static constexpr bool scaled = false;
    static constexpr bool uv = false;
    static constexpr unsigned bytes = 4;
};
template <>
struct Store<WAVE_F16> {
    static constexpr bool scaled = true;
    static constexpr bool uv = false;
    static constexpr unsigned bytes = 2;
    static __device__ __forceinline__ float dec(unsigned bits)
    {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)bits);
    }
    static __device__ __forceinline__ unsigned enc(float x)
    {
        return __builtin_bit_cast(unsigned short, (_Float16)x);
    }
    // two values packed low, high: one packed conversion (round to nearest
    // even, as the scalar one) instead of two
    static __device__ __forceinline__ unsigned enc2(float lo, float hi)
    {
        typedef float f2v __attribute__((ext_vector_type(2)));
        typedef _Float16 h2v __attribute__((ext_vector_type(2)));
        const f2v f = {lo, hi};
        return __builtin_bit_cast(unsigned, __builtin_convertvector(f, h2v));
    }
};
template <>
struct Store<WAVE_BF16> {
    static constexpr bool scaled = true;
    static constexpr bool uv = false;
    static constexpr unsigned bytes = 2;
    static __device__ __forceinline__ float dec(unsigned bits) { return __uint_as_float(bits << 16); }
    static __device__ __forceinline__ unsigned enc(float x)
    {
        return __builtin_bit_cast(unsigned short, (__bf16)x);
    }
    static __device__ __forceinline__ unsigned enc2(float lo, float hi) { return enc(lo) | (enc(hi) << 16); }
};
// u and its step change d = u^n - u^{n-1}, same 16-bit encodings
template <>
struct Store<WAVE_F16_UV> : Store<WAVE_F16> {
    static constexpr bool uv = true;
};
template <>
struct Store<WAVE_BF16_UV> : Store<WAVE_BF16> {
    static constexpr bool uv = true;
};

// Raw buffer access.  A buffer resource covers one plane of one field; any
// byte offset at or past its size reads as zero and drops stores, which is
// how out-of-range tile cells are masked without branches.
typedef unsigned u4raw __attribute__((vector_size(16)));
typedef unsigned u2raw __attribute__((vector_size(8)));
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw (stride 0) access
constexpr unsigned kOff = 0xffffffffu;  // an offset outside every resource

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *field, long long plane_bytes,
                                                            int z)
{
    const char *p = reinterpret_cast<const char *>(field) + (long long)(z + kGhost) * plane_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, (int)plane_bytes,
                                             kRsrcWord3);
}

// The same for a plane the stencil may reach outside the grid (z < 0 or
// z >= nz): a ghost plane gets an empty resource, so its loads return the
// zeros it holds without reading memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stencil_plane_rsrc(const void *field, long long plane_bytes,
                                                                    int z, int nz)
{
    const char *p = reinterpret_cast<const char *>(field) + (long long)(z + kGhost) * plane_bytes;
    const int size = (z >= 0 && z < nz) ? (int)plane_bytes : 0;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, size, kRsrcWord3);
}

// Cache policy of a buffer access (gfx950 encoding of the aux operand):
// bit 1 = non-temporal.  u^{n-1} and k are read exactly once per step and
// u^{n+1} is not read again in the step, so they are streamed
// non-temporally; u^n is read by the neighbouring tiles as their halo and
// keeps the default policy, so it stays resident in L2.
typedef double dv2 __attribute__((ext_vector_type(2)));

constexpr int kKeep = 0;
constexpr int kStream = 2;
// device scope (sc1): the load misses the CU's L1 and is served by the L2,
// so it sees what other CUs of the same XCD stored (their stores have
// reached the L2 before they signal completion)
constexpr int kCoh = 16;

// Four consecutive cells as stored (16 bytes of FP32, 8 bytes of 16-bit
// values), and decoded to FP32 (times `scale` for 16-bit data).  Values
// loaded ahead of their use are held raw, so that a 16-bit prefetch holds
// half the registers of its decoded form.
template <int KIND>
using Raw4 = std::conditional_t<KIND == WAVE_F32, u4raw, u2raw>;

template <int KIND, int POL>
__device__ __forceinline__ Raw4<KIND> load_raw4(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (KIND == WAVE_F32)
        return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, POL);
    else
        return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, POL);
}

template <int KIND>
__device__ __forceinline__ f4 decode4(const Raw4<KIND> &v, float scale = 1.f)
{
    f4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if constexpr (KIND == WAVE_F32)
            o.v[e] = __uint_as_float(v[e]);
        else
            o.v[e] = Store<KIND>::dec((v[e >> 1] >> (16 * (e & 1))) & 0xffffu) * scale;
    }
    return o;
}

template <int KIND, int POL>
__device__ __forceinline__ f4 load4(__amdgpu_buffer_rsrc_t r, unsigned off, float scale)
{
    return decode4<KIND>(load_raw4<KIND, POL>(r, off), scale);
}

template <int KIND>
__device__ __forceinline__ void store4(__amdgpu_buffer_rsrc_t r, unsigned off, const f4 &v, float inv)
{
    if constexpr (KIND == WAVE_F32) {
        u4raw w;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            w[e] = __float_as_uint(v.v[e]);
        __builtin_amdgcn_raw_buffer_store_b128(w, r, off, 0, kStream);
    } else {
        u2raw w;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            w[h] = Store<KIND>::enc2(v.v[2 * h] * inv, v.v[2 * h + 1] * inv);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, kStream);
    }
}

// Element read outside the hot loop (receivers, exports).
template <int KIND>
__device__ __forceinline__ float read_elem(const void *f, long long i, float scale)
{
    if constexpr (KIND == WAVE_F32)
        return static_cast<const float *>(f)[i];
    else
        return Store<KIND>::dec(static_cast<const unsigned short *>(f)[i]) * scale;
}

// Scales of one step with 16-bit storage.  u^{n+1} is bounded by
// 7 max(|u^n|, |u^{n-1}|) + |s_n| (2 + 1 from the time levels, 4 from
// k |lap| under the stability limit, G <= 1); its exponent is chosen so
// that 8 M + |s_n| < 2^(e + 14), which leaves a factor 4 below the FP16
// maximum.  All work-groups compute the same value from the same inputs.
struct Scales {
    float cur, prev, out_inv, out;
    int e_out;
};

// The same step in the stored (scaled) units.  With U, P, K the decoded
// but unscaled u^n, u^{n-1}, k and every scale a power of two, the stored
// u^{n+1} is
//   O = g (fma(K, LAP_C(U), 2A U) - g B P),
//   A = sc_cur / sc_out, B = sc_prev / sc_out, C = k_scale * A,
// with LAP_C the Laplacian whose weights are multiplied by C.  Scaling by
// a power of two commutes with every FP32 rounding, so this is bit for bit
// the decode -> compute -> encode sequence, without the per-value
// multiplies.
//
// With u-and-change storage the second input is D, the stored d^n =
// u^n - u^{n-1} (exponent one above u^n's), and u^{n-1} in output units is
// A U - B D with B = sc_d / sc_out; the same expression follows.  The new
// change d^{n+1} = u^{n+1} - u^n is formed in FP32 before either is
// rounded and stored with the exponent of u^{n+1} plus one (it is bounded
// by |u^{n+1}| + |u^n| < 2^(e + 15)).
struct Folded {
    Coefs c;       // weights times C
    float two_a;   // 2 A
    float b;       // B
    float a;       // A
};

__device__ __forceinline__ Folded fold_scales(const Coefs &c, const Scales &sc, float k_scale)
{
    Folded f;
    const float A = sc.cur * sc.out_inv;
    const float C = k_scale * A;
    f.c.ctr = c.ctr * C;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        f.c.cx[m] = c.cx[m] * C;
        f.c.cy[m] = c.cy[m] * C;
        f.c.cz[m] = c.cz[m] * C;
    }
    f.two_a = 2.f * A;
    f.b = sc.prev * sc.out_inv;
    f.a = A;
    return f;
}

template <int KIND>
__device__ __forceinline__ Scales step_scales(const StepArgs &a)
{
    const int n = a.step;
    const float m = fmaxf(__uint_as_float(a.maxes[n & 3]), __uint_as_float(a.maxes[(n + 3) & 3]));
    const float s = a.src_z >= 0 ? fabsf(src_value(a)) : 0.f;
    const float bound = 8.f * m + s;
    int e = 0;
    if (bound > 0.f && bound < INFINITY) {
        int ex;
        (void)frexpf(bound, &ex);  // bound < 2^ex
        e = min(max(ex - kScaledTopExp, -110), 110);
    }
    Scales sc;
    sc.cur = ldexpf(1.f, a.exps[n & 3]);
    // second input: u^{n-1}, or d^n (exponent of u^n plus one)
    sc.prev = Store<KIND>::uv ? ldexpf(1.f, a.exps[n & 3] + 1) : ldexpf(1.f, a.exps[(n + 3) & 3]);
    sc.out = ldexpf(1.f, e);
    sc.out_inv = ldexpf(1.f, -e);
    sc.e_out = e;
    return sc;
}

// Publish this step's exponent and clear the max slot the next step fills
// after this one (slot n + 2, which no launch of this step reads).
__device__ __forceinline__ void publish_scale(const StepArgs &a, const Scales &sc, int lid, int tid)
{
    if (lid == 0 && tid == 0) {
        a.exps[(a.step + 1) & 3] = sc.e_out;
        a.maxes[(a.step + 2) & 3] = 0u;
    }
}

// Fold a per-thread max |u^{n+1}| into the step's slot: a reduction across
// the wave, then one atomic per wave (on the float bit pattern, valid for
// non-negative values).
__device__ __forceinline__ void fold_max(const StepArgs &a, float m)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        m = fmaxf(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0)
        atomicMax(&a.maxes[(a.step + 1) & 3], __float_as_uint(m));
}

// Receiver epilogue: after the whole tile column is written, copy the
// receivers this work-group owns into the trace row.
template <int KIND>
__device__ __forceinline__ void sample_receivers(const StepArgs &a, int lid, int tid, int nt,
                                                 float scale)
{
    if (!a.trace_row)
        return;
    const int r0 = a.rec_start[lid], r1 = a.rec_start[lid + 1];
    if (r0 == r1)
        return;
    __syncthreads();
    for (int i = r0 + tid; i < r1; i += nt)
        a.trace_row[a.rec_idx[i]] = read_elem<KIND>(a.out, a.rec_off[i], scale);
}

// Calls f(integral_constant<int, S>) for S = B, B+1, ... < E while f
// returns true: a loop unrolled at compile time, so every index that
// depends on S is a constant and register arrays stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for_while(F &&f)
{
    if constexpr (B < E) {
        if (f(std::integral_constant<int, B>{}))
            static_for_while<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// the step

// One work-group's share of a step: the tile and z-chunk numbered `lid`
// (tiles x fastest, then y, then chunks) of the grid described by `a`.
template <int KIND, int TXV, int TY, int RY, int MODE = kFwd, bool COH = false, bool CACHED = false>
__device__ __forceinline__ void tile_step(const StepArgs &a, int lid)
{
    constexpr int NT = TXV * TY;
    constexpr int TYR = TY * RY;             // tile rows
    constexpr int LW = TXV + 2;              // float4 per LDS row: one halo float4 each side
    constexpr int LH = TYR + 8;              // LDS rows: 4 halo rows each side
    constexpr int NH = 8 * TXV + 2 * TYR;    // halo float4 per plane
    constexpr int HPT = (NH + NT - 1) / NT;  // halo float4 per thread
    constexpr int QS = 10;                   // queue slots: 9 live planes + 1 being filled
    constexpr unsigned EB = Store<KIND>::bytes;
    constexpr bool SCALED = Store<KIND>::scaled;
    constexpr bool UV = Store<KIND>::uv;          // second input is d^n, also written
    constexpr bool FUS = MODE == kFus;            // adjoint step + imaging term of the step after it
    constexpr bool ADJ = MODE == kAdj || FUS;     // the stencil field is phi, scaled by G on load
    constexpr bool IMG = MODE == kImg;
    constexpr bool GRAD = IMG || FUS;             // adds an imaging term to the FP64 accumulator
    static_assert(MODE == kFwd || KIND == WAVE_F32, "adjoint and imaging steps are FP32 only");
    // load policies of the wave fields (k never changes during a run);
    // CACHED: u^{n-1} and k too keep the default policy, for grids whose
    // fields fit in the memory-side cache together.  The step change d^n of
    // the u-and-change forms keeps it too: with the z-march reversed every
    // launch, the d planes one launch touches last are the next one's first,
    // and the memory-side cache serves part of them (512^3: FP16 513 -> 526,
    // BF16 519 -> 546 Gpts/s; also keeping k was slower, and so was keeping
    // u^{n-1} and k in the two-level forms)
    constexpr int PK = kKeep | (COH ? kCoh : 0);
    constexpr int PS = ((CACHED || UV) ? kKeep : kStream) | (COH ? kCoh : 0);
    constexpr int PKK = CACHED ? kKeep : kStream;
    __shared__ f4 lds[2][LH][LW];
    // second stencil field (the forward level of the imaging term), fused mode only
    __shared__ f4 lds2[FUS ? 2 : 1][FUS ? LH : 1][FUS ? LW : 1];

    const int tx = lid % a.ntx;
    const int rest = lid / a.ntx;
    const int ty = rest % a.nty;
    const int ch = rest / a.nty;
    const int z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, a.nz);
    // the chunk's planes in march order: march position l is plane zp(l)
    // (positions -4 .. -1 and len .. len + 3 are the chunk's z halo)
    const int len = z1 - z0;
    const bool down = a.zdown & 1;
    auto zp = [&](int l) { return down ? z1 - 1 - l : z0 + l; };

    const int tid = threadIdx.x;
    const int lx = tid % TXV;
    const int ly = tid / TXV;
    const int xq0 = tx * TXV;          // first 4-cell column of the tile
    const int y0 = ty * TYR;           // first row of the tile
    const int xq = xq0 + lx;           // this thread's 4-cell column
    const int x = 4 * xq;

    Scales sc{1.f, 1.f, 1.f, 1.f, 0};
    Folded fd{a.c, 2.f, 1.f, 1.f};
    if constexpr (SCALED) {
        sc = step_scales<KIND>(a);
        publish_scale(a, sc, lid, tid);
        fd = fold_scales(a.c, sc, a.k_scale);
    }

    // Only 4-cell groups holding interior cells are read (the ragged last
    // group's right-ghost lanes with them); ghost rows, columns and planes
    // hold zero, and their loads are masked so that they return zero without
    // reading memory.
    const bool col_interior = x < a.nx;
    const bool col_full = x + 3 < a.nx;

    // own rows: byte offsets within a plane (kOff when masked)
    int row[RY];
    bool row_int[RY];
    unsigned own_ld[RY], own_in[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = y0 + ly * RY + r;
        row_int[r] = col_interior && row[r] < a.ny;
        const unsigned b = EB * unsigned((row[r] + kGhost) * a.px + a.x0 + x);
        own_in[r] = row_int[r] ? b : kOff;
        own_ld[r] = own_in[r];
    }

    // halo items of this thread
    unsigned h_b[HPT];
    int h_lds[HPT];  // flat LDS index (row * LW + col), -1 when unused
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
        const int i = tid + h * NT;
        int hr, hc;
        if (i < 8 * TXV) {
            const int band = i / TXV;
            hr = band < 4 ? band - 4 : TYR + band - 4;
            hc = i % TXV;
        } else {
            const int j = i - 8 * TXV;
            hr = j % TYR;
            hc = (j / TYR) ? TXV : -1;
        }
        const bool use = i < NH;
        h_lds[h] = use ? (hr + 4) * LW + (hc + 1) : -1;
        const int gy = y0 + hr;
        const int gq = xq0 + hc;
        const bool ok = use && gy >= 0 && gy < a.ny && gq >= 0 && gq < a.nxq;
        h_b[h] = ok ? EB * unsigned((gy + kGhost) * a.px + a.x0 + 4 * gq) : kOff;
    }
    // adjoint: sponge factor g_x g_y of every cell this thread loads
    // (cells outside the interior hold zeros; their factor is irrelevant)
    f4 gh[ADJ ? HPT : 1];
    if constexpr (ADJ) {
#pragma unroll
        for (int h = 0; h < HPT; ++h) {
            const int i = tid + h * NT;
            int hr, hc;
            if (i < 8 * TXV) {
                const int band = i / TXV;
                hr = band < 4 ? band - 4 : TYR + band - 4;
                hc = i % TXV;
            } else {
                const int j = i - 8 * TXV;
                hr = j % TYR;
                hc = (j / TYR) ? TXV : -1;
            }
            const int gy = y0 + hr;
            const float fy = (gy >= 0 && gy < a.ny) ? a.gy[gy] : 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gxi = 4 * (xq0 + hc) + e;
                gh[h].v[e] = (gxi >= 0 && gxi < a.nx) ? a.gx[gxi] * fy : 0.f;
            }
        }
    }

    // sponge factors that do not change along z
    f4 gxv = {{1.f, 1.f, 1.f, 1.f}};
    if (col_interior) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            gxv.v[e] = (x + e < a.nx) ? a.gx[x + e] : 1.f;
    }
    float gyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r)
        gyv[r] = row_int[r] ? a.gy[row[r]] : 1.f;
    f4 gown[ADJ ? RY : 1];  // adjoint: g_x g_y of the own cells
    if constexpr (ADJ) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gown[r].v[e] = gxv.v[e] * gyv[r];
    }

    // source ownership (the value is read once, before the march)
    int src_r = -1, src_e = 0;
    if (a.src_z >= z0 && a.src_z < z1 && (a.src_x >> 2) == xq) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (row[r] == a.src_y)
                src_r = r;
        src_e = a.src_x & 3;
    }
    const float sval = src_r >= 0 ? src_value(a) * sc.out_inv : 0.f;

    const long long pbytes = a.plane * (long long)EB;
    const __amdgpu_buffer_rsrc_t gz_r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(a.gz), (short)0, a.nz * (int)sizeof(float), kRsrcWord3);

    // register queue: at phase s the plane of march position l - 4 + i
    // lives in slot (s + i) % QS
    auto gz_at = [&](int z) {  // g_z, zero outside the interior (reads nothing there)
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(gz_r, 4u * unsigned(z), 0, 0));
    };
    f4 q[QS][RY];
    f4 q2[FUS ? QS : 1][RY];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int zi = zp(i - 4);
        const __amdgpu_buffer_rsrc_t rc = stencil_plane_rsrc(a.cur, pbytes, zi, a.nz);
#pragma unroll
        for (int r = 0; r < RY; ++r)
            q[i][r] = load4<KIND, PK>(rc, own_ld[r], 1.f);
        if constexpr (FUS) {
            const __amdgpu_buffer_rsrc_t ra = stencil_plane_rsrc(a.aux, pbytes, zi, a.nz);
#pragma unroll
            for (int r = 0; r < RY; ++r)
                q2[i][r] = load4<KIND, PK>(ra, own_ld[r], 1.f);
        }
        if constexpr (ADJ) {
            const float gzi = gz_at(zi);
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    q[i][r].v[e] = mul_rounded(q[i][r].v[e], gown[r].v[e] * gzi);
        }
    }

    // values of the next plane, loaded one plane ahead into the set of the
    // other parity (no copies, so no wait before the next loads are issued)
    Raw4<KIND> pv[2][RY], kv[2][RY], hv[2][HPT];
    f4 hv2[FUS ? 2 : 1][FUS ? HPT : 1];
    float gzv[2], gzq[2];  // g_z of the plane and (adjoint) of the queue plane four positions on
    auto prefetch = [&](int l, int slot, int set) {
        const int z = zp(l), zq = zp(l + 4);
        const __amdgpu_buffer_rsrc_t rq = stencil_plane_rsrc(a.cur, pbytes, zq, a.nz);
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(UV ? a.dlt : a.nxt, pbytes, z);
        const __amdgpu_buffer_rsrc_t rk = plane_rsrc(a.k, pbytes, z);
        const __amdgpu_buffer_rsrc_t rh = plane_rsrc(a.cur, pbytes, z);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[slot][r] = load4<KIND, PK>(rq, own_ld[r], 1.f);
            pv[set][r] = load_raw4<KIND, PS>(rp, own_in[r]);
            kv[set][r] = load_raw4<KIND, PKK>(rk, own_in[r]);
        }
#pragma unroll
        for (int h = 0; h < HPT; ++h)
            hv[set][h] = load_raw4<KIND, PK>(rh, h_b[h]);
        if constexpr (FUS) {
            const __amdgpu_buffer_rsrc_t raq = stencil_plane_rsrc(a.aux, pbytes, zq, a.nz);
            const __amdgpu_buffer_rsrc_t rah = plane_rsrc(a.aux, pbytes, z);
#pragma unroll
            for (int r = 0; r < RY; ++r)
                q2[slot][r] = load4<KIND, PK>(raq, own_ld[r], 1.f);
#pragma unroll
            for (int h = 0; h < HPT; ++h)
                hv2[set][h] = load4<KIND, PK>(rah, h_b[h], 1.f);
        }
        gzv[set] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(gz_r, 4u * z, 0, 0));
        if constexpr (ADJ)
            gzq[set] = gz_at(zq);
    };
    prefetch(0, 8, 0);

    float tmax = 0.f;  // max |stored u^{n+1}| written by this thread (16-bit storage)
    const Coefs c = fd.c;
    for (int lb = 0; lb < len; lb += QS) {
        static_for_while<0, QS>([&](auto phase) __attribute__((always_inline)) -> bool {
            constexpr int s = decltype(phase)::value;
            const int l = lb + s;
            if (l >= len)
                return false;
            const int z = zp(l);
            const int cur_set = s & 1;
            // next plane (clamped on the last one, whose loads go unused)
            prefetch(min(l + 1, len - 1), (s + 9) % QS, cur_set ^ 1);
            // imaging modes: this plane's accumulator values, loaded before
            // the arithmetic so that their latency overlaps it.  Each cell is
            // read and written once per step, but with the z-march reversed
            // every launch the planes a launch touches last are the first
            // the next one touches, so the accumulator keeps the default
            // cache policy and the memory-side cache serves part of it
            dv2 gacc[GRAD ? RY : 1][2] = {};
            if constexpr (GRAD) {
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    if (col_full && row_int[r]) {
                        const dv2 *gp = reinterpret_cast<const dv2 *>(
                            a.grad + (long long)(z + kGhost) * a.plane + own_in[r] / EB);
                        gacc[r][0] = gp[0];
                        gacc[r][1] = gp[1];
                    }
            }

            if constexpr (ADJ) {
                // psi = G phi: the plane that just entered the queue (four positions on)
                // and this plane's halo
#pragma unroll
                for (int r = 0; r < RY; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        q[(s + 8) % QS][r].v[e] =
                            mul_rounded(q[(s + 8) % QS][r].v[e], gown[r].v[e] * gzq[cur_set]);
            }
            const int b = l & 1;
            f4 *L = &lds[b][0][0];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                L[(4 + ly * RY + r) * LW + lx + 1] = q[(s + 4) % QS][r];
#pragma unroll
            for (int h = 0; h < HPT; ++h) {
                f4 hd = decode4<KIND>(hv[cur_set][h]);
                if constexpr (ADJ) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        hd.v[e] = mul_rounded(hd.v[e], gh[h].v[e] * gzv[cur_set]);
                }
                if (h_lds[h] >= 0)
                    L[h_lds[h]] = hd;
            }
            f4 *L2 = &lds2[FUS ? b : 0][0][0];
            if constexpr (FUS) {
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    L2[(4 + ly * RY + r) * LW + lx + 1] = q2[(s + 4) % QS][r];
#pragma unroll
                for (int h = 0; h < HPT; ++h)
                    if (h_lds[h] >= 0)
                        L2[h_lds[h]] = hv2[cur_set][h];
            }
            __syncthreads();

            // y taps: LDS rows ly*RY - 4 .. ly*RY + RY + 3 of this column,
            // own rows straight from the queue
            f4 ycol[RY + 8];
#pragma unroll
            for (int j = 0; j < RY + 8; ++j) {
                if (j >= 4 && j < 4 + RY)
                    ycol[j] = q[(s + 4) % QS][j - 4];
                else
                    ycol[j] = L[(ly * RY + j) * LW + lx + 1];
            }
            f4 ycol2[FUS ? RY + 8 : 1];
            if constexpr (FUS) {
#pragma unroll
                for (int j = 0; j < RY + 8; ++j) {
                    if (j >= 4 && j < 4 + RY)
                        ycol2[j] = q2[(s + 4) % QS][j - 4];
                    else
                        ycol2[j] = L2[(ly * RY + j) * LW + lx + 1];
                }
            }

            const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.out, pbytes, z);
            const __amdgpu_buffer_rsrc_t rdl = plane_rsrc(UV ? a.dlt : a.out, pbytes, z);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const f4 pvd = decode4<KIND>(pv[cur_set][r]);
                const f4 kvd = decode4<KIND>(kv[cur_set][r]);
                const f4 xl = L[(4 + ly * RY + r) * LW + lx];
                const f4 xr = L[(4 + ly * RY + r) * LW + lx + 2];
                const f4 ctr = q[(s + 4) % QS][r];
                float xs[12];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xs[e] = xl.v[e];
                    xs[4 + e] = ctr.v[e];
                    xs[8 + e] = xr.v[e];
                }
                float xs2[FUS ? 12 : 1];
                if constexpr (FUS) {
                    const f4 xl2 = L2[(4 + ly * RY + r) * LW + lx];
                    const f4 xr2 = L2[(4 + ly * RY + r) * LW + lx + 2];
                    const f4 ctr2 = q2[(s + 4) % QS][r];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        xs2[e] = xl2.v[e];
                        xs2[4 + e] = ctr2.v[e];
                        xs2[8 + e] = xr2.v[e];
                    }
                }
                f4 out, img;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float lap;
                    if constexpr (SCALED) {
                        lap = c.ctr * ctr.v[e];
#pragma unroll
                        for (int m = 1; m <= 4; ++m) {
                            lap = fmaf(c.cx[m - 1], xs[4 + e + m] + xs[4 + e - m], lap);
                            lap = fmaf(c.cy[m - 1], ycol[4 + r + m].v[e] + ycol[4 + r - m].v[e], lap);
                            lap = fmaf(c.cz[m - 1],
                                       q[(s + 4 + m) % QS][r].v[e] + q[(s + 4 - m + QS) % QS][r].v[e],
                                       lap);
                        }
                    } else {
                        const float u2 = 2.f * ctr.v[e];
                        lap = 0.f;
#pragma unroll
                        for (int m = 1; m <= 4; ++m) {
                            lap = fmaf(c.cx[m - 1], (xs[4 + e + m] + xs[4 + e - m]) - u2, lap);
                            lap = fmaf(c.cy[m - 1], (ycol[4 + r + m].v[e] + ycol[4 + r - m].v[e]) - u2,
                                       lap);
                            lap = fmaf(c.cz[m - 1],
                                       (q[(s + 4 + m) % QS][r].v[e] + q[(s + 4 - m + QS) % QS][r].v[e]) -
                                           u2,
                                       lap);
                        }
                    }
                    const float g = gxv.v[e] * gyv[r] * gzv[cur_set];
                    if constexpr (IMG) {
                        // imaging term (G phi / k) lap a
                        out.v[e] = (g * pvd.v[e]) / kvd.v[e] * lap;
                    } else if constexpr (ADJ) {
                        const float t = fmaf(kvd.v[e], lap, 2.f * ctr.v[e]);
                        out.v[e] = fmaf(-g * g, pvd.v[e], t);
                        if constexpr (FUS) {
                            // imaging term of the step after this one: the
                            // centre already holds G phi, bit for bit g * phi
                            const float u2b = 2.f * xs2[4 + e];
                            float lap2 = 0.f;
#pragma unroll
                            for (int m = 1; m <= 4; ++m) {
                                lap2 = fmaf(c.cx[m - 1], (xs2[4 + e + m] + xs2[4 + e - m]) - u2b, lap2);
                                lap2 = fmaf(c.cy[m - 1],
                                            (ycol2[4 + r + m].v[e] + ycol2[4 + r - m].v[e]) - u2b, lap2);
                                lap2 = fmaf(c.cz[m - 1],
                                            (q2[(s + 4 + m) % QS][r].v[e] + q2[(s + 4 - m + QS) % QS][r].v[e]) -
                                                u2b,
                                            lap2);
                            }
                            img.v[e] = ctr.v[e] / kvd.v[e] * lap2;
                        }
                    } else {
                        float t, pe;
                        if constexpr (SCALED) {
                            t = fmaf(kvd.v[e], lap, fd.two_a * ctr.v[e]);
                            if constexpr (UV)  // u^{n-1} = u^n - d^n
                                pe = fmaf(-fd.b, pvd.v[e], fd.a * ctr.v[e]);
                            else
                                pe = fd.b * pvd.v[e];
                        } else {
                            t = fmaf(kvd.v[e], lap, 2.f * ctr.v[e]);
                            pe = pvd.v[e];
                        }
                        t = fmaf(-g, pe, t);
                        out.v[e] = g * t;
                    }
                }
                // the accumulator has the field layout with 8-byte cells, so
                // a full 4-cell group is two aligned 16-byte pairs
                auto add_grad = [&](const f4 &t) __attribute__((always_inline)) {
                    if (col_full) {
                        if (row_int[r]) {
                            dv2 *gp = reinterpret_cast<dv2 *>(a.grad + (long long)(z + kGhost) * a.plane +
                                                              own_in[r] / EB);
                            dv2 g0 = gacc[r][0], g1 = gacc[r][1];
                            g0.x += (double)t.v[0];
                            g0.y += (double)t.v[1];
                            g1.x += (double)t.v[2];
                            g1.y += (double)t.v[3];
                            gp[0] = g0;
                            gp[1] = g1;
                        }
                    } else if (row_int[r]) {
                        double *gp = a.grad + (long long)(z + kGhost) * a.plane + own_in[r] / EB;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (x + e < a.nx)
                                gp[e] += (double)t.v[e];
                    }
                };
                if constexpr (IMG) {
                    add_grad(out);
                    continue;
                }
                if constexpr (FUS)
                    add_grad(img);
                if (src_r == r && z == a.src_z) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e == src_e)
                            out.v[e] += sval;
                }
                f4 dn;  // d^{n+1} in its own units (u-and-change storage)
                if constexpr (UV) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        dn.v[e] = 0.5f * (out.v[e] - fd.a * ctr.v[e]);
                }
                // In a ragged last group the cells past nx are right-ghost
                // cells, which hold zero: writing zero there keeps them so and
                // lets the group go out as one whole store (no partial writes).
                if (!col_full) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (x + e >= a.nx) {
                            out.v[e] = 0.f;
                            if constexpr (UV)
                                dn.v[e] = 0.f;
                        }
                }
                store4<KIND>(ro, own_in[r], out, 1.f);
                if constexpr (UV)
                    store4<KIND>(rdl, own_in[r], dn, 1.f);
                if constexpr (SCALED) {
                    if (row_int[r]) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            tmax = fmaxf(tmax, fabsf(out.v[e]));
                    }
                }
            }
            return true;
        });
    }

    if constexpr (SCALED)
        fold_max(a, tmax * sc.out);
    sample_receivers<KIND>(a, lid, tid, NT, sc.out);
}

template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_tiled(StepArgs a)
{
    const int lid = logical_wg();
    if (lid >= a.nwg)
        return;
    tile_step<KIND, TXV, TY, RY>(a, lid);
}

// The FP32 step with every field read with the default cache policy: for
// grids whose three fields fit in the GPU's memory-side cache together, so
// that u^{n-1} and k, read once per step, are still cached at the next step
// (the host picks it; same arithmetic as step_tiled).
template <int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_tiled_cached(StepArgs a)
{
    const int lid = logical_wg();
    if (lid >= a.nwg)
        return;
    tile_step<WAVE_F32, TXV, TY, RY, kFwd, false, true>(a, lid);
}

template <int MODE, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void adjoint_tiled(StepArgs a)
{
    const int lid = logical_wg();
    if (lid >= a.nwg)
        return;
    tile_step<WAVE_F32, TXV, TY, RY, MODE>(a, lid);
}




// ---------------------------------------------------------------------------
// many shots per launch


// The items of one time step j of every shot in a group: work-group b runs
// on XCD b % 8 (blocks are dealt to the XCDs round-robin) and takes items
// of that XCD's range by atomic ticket until the range is exhausted, so
// long and short items balance dynamically while neighbouring tiles still
// share an XCD's L2.  Step j draws from counter set j & 1 and clears set
// (j + 1) & 1 for the next step, which starts only after this one has ended
// (a launch boundary, or a grid barrier in the single-launch run).
template <int KIND, int TXV, int TY, int RY>
__device__ __forceinline__ void batch_step_items(const ShotDesc *__restrict__ shots, const BatchItems &it, int j,
                                                 int &ticket)
{
    const int xcd = blockIdx.x & 7;
    int *cnt = it.counters + 8 * (j & 1);
    if (blockIdx.x == 0 && threadIdx.x < 8)
        it.counters[8 * ((j + 1) & 1) + threadIdx.x] = 0;
    const int first = it.xcd_start[xcd], last = it.xcd_start[xcd + 1];
    for (;;) {
        if (threadIdx.x == 0)
            ticket = atomicAdd(&cnt[xcd], 1);
        __syncthreads();
        const int item = first + ticket;
        __syncthreads();  // all threads have read the ticket (and left the LDS of the last item)
        if (item >= last)
            break;
        const ShotDesc &d = shots[it.shot[item]];
        StepArgs a = d.a;
        if (j & 1) {
            const void *t = a.cur;
            a.cur = a.nxt;
            a.nxt = const_cast<void *>(t);
        }
        a.out = a.nxt;  // in place
        const int n = d.n0 + j;
        a.step = n & 0x3fffffff;
        a.zdown = n & 1;
        a.trace_row = d.traces ? d.traces + (size_t)n * d.nrec : nullptr;
        a.src_ptr = d.src ? d.src + j : nullptr;
        a.src_val = 0.f;
        if (!d.src)
            a.src_z = -1;  // no source values given: no injection
        tile_step<KIND, TXV, TY, RY>(a, it.lid[item]);
    }
}

// One time step of every shot in a group as a persistent launch: the grid
// holds as many work-groups as fit on the GPU at once.
template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_batch(const ShotDesc *__restrict__ shots,
                                                       BatchItems it, int j)
{
    __shared__ int ticket;
    batch_step_items<KIND, TXV, TY, RY>(shots, it, j, ticket);
}

// Every step of a run of every shot in a group in one cooperative launch
// (all work-groups resident at once).  Each step is the work of step_batch;
// a grid-wide barrier replaces the launch boundary between steps.  Before
// a work-group arrives, its stores are made visible device-wide: every
// thread waits for its own stores to complete, then thread 0 arrives with an
// agent-scope release (which writes back its XCD's L2).  It leaves after an
// agent-scope acquire, so a step reads what the step before wrote on any
// XCD.  Every wait is bounded by a wall-clock limit and a shared abort flag:
// a wait that runs past the limit raises the flag, every work-group stops
// at its next barrier, and the host reports the run as failed.
template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_batch_run(const ShotDesc *__restrict__ shots, BatchItems it,
                                                           RunSync rs)
{
    __shared__ int ticket;
    __shared__ int stop;
    const unsigned long long deadline = wall_clock64() + rs.timeout;
    unsigned gen = 0;  // barriers this work-group has passed
    for (int jj = 0; jj < rs.nsteps; ++jj) {
        batch_step_items<KIND, TXV, TY, RY>(shots, it, rs.j0 + jj, ticket);
        if (jj + 1 == rs.nsteps)
            break;  // the launch boundary orders the last step
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
        __syncthreads();
        if (threadIdx.x == 0) {
            stop = 0;
            const unsigned arrived =
                __hip_atomic_fetch_add(rs.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived + 1 == gridDim.x) {
                // the last to arrive opens the barrier for everyone
                __hip_atomic_store(rs.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(rs.gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                while (__hip_atomic_load(rs.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    if (wall_clock64() > deadline ||
                        __hip_atomic_load(rs.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_store(rs.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        stop = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ++gen;
        }
        __syncthreads();
        if (stop)
            return;
    }
}

// Schedule 2 (switched off in the host code; see there): every step of
// every shot of a group in one launch (FP32).
// A work item is (step j, shot, tile, z-chunk).  The shots are pinned to
// XCDs (blocks with equal b mod 8 run on one XCD; which one depends on the
// launches before), so producers and consumers of a
// shot's fields share one L2; each XCD hands out its items by ticket in
// step order.  An item of step j starts when its own tile/chunk and the
// tiles and chunks its stencil reads from have completed step j - 1, which
// also means none of them still reads the buffer the item overwrites.  A
// work-group only waits for items with lower tickets, which running
// work-groups hold, so the waits always end; each wait is still bounded
// (FlowPlan::wait_limit polls), and a wait that gives up raises the abort
// flag, on which every work-group stops at its next check.

// Whether every item that item (j, lid) of shot fs depends on has completed
// step j - 1 (steps counted from the launch's first step).
__device__ __forceinline__ bool flow_ready(const FlowPlan &p, const FlowShot &fs, int lid, int j)
{
    if (j == 0)
        return true;
    if (p.wait_limit < 0)  // failure-path hook: every wait gives up
        return false;
    const int tiles = fs.ntx * fs.nty;
    const int tx = lid % fs.ntx, ty = (lid / fs.ntx) % fs.nty, ch = lid / tiles;
    const int *done = p.done + fs.done;
    int polls = 0;
    auto wait_for = [&](int l) -> bool {
        while (__hip_atomic_load(done + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < j) {
            if (polls >= p.wait_limit || __hip_atomic_load(p.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return false;
            ++polls;
            __builtin_amdgcn_s_sleep(2);
        }
        return true;
    };
    const int c0 = max(0, ch - fs.zreach), c1 = min(fs.nch - 1, ch + fs.zreach);
    for (int c = c0; c <= c1; ++c)
        if (!wait_for(c * tiles + ty * fs.ntx + tx))
            return false;
    const int base = ch * tiles;
    if (tx > 0 && !wait_for(base + ty * fs.ntx + tx - 1))
        return false;
    if (tx + 1 < fs.ntx && !wait_for(base + ty * fs.ntx + tx + 1))
        return false;
    if (ty > 0 && !wait_for(base + (ty - 1) * fs.ntx + tx))
        return false;
    if (ty + 1 < fs.nty && !wait_for(base + (ty + 1) * fs.ntx + tx))
        return false;
    return true;
}

template <int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_flow(const ShotDesc *__restrict__ shots, FlowPlan p)
{
    __shared__ int item[3];  // step, FlowShot index, tile/chunk; step < 0: stop
    const int xcd = blockIdx.x & 7;
    const int per = p.xcd_items[xcd];
    const int total = per * p.nsteps;
    for (;;) {
        if (threadIdx.x == 0) {
            int j = -1, k = 0, lid = 0;
            const int t = atomicAdd(&p.tickets[xcd], 1);
            if (t < total && !__hip_atomic_load(p.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                j = t / per;
                const int r = t - j * per;
                k = p.xcd_shot[xcd];
                while (k + 1 < p.xcd_shot[xcd + 1] && r >= p.shots[k].base + p.shots[k].items)
                    ++k;
                lid = r - p.shots[k].base;
                if (!flow_ready(p, p.shots[k], lid, j)) {
                    __hip_atomic_store(p.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    j = -1;
                }
            }
            item[0] = j;
            item[1] = k;
            item[2] = lid;
        }
        __syncthreads();
        const int j = item[0], k = item[1], lid = item[2];
        __syncthreads();  // all threads have read the item (and left the LDS of the last one)
        if (j < 0)
            break;
        const FlowShot &fs = p.shots[k];
        const ShotDesc &d = shots[fs.desc];
        const int jj = p.j0 + j;  // step within the run
        StepArgs a = d.a;
        if (jj & 1) {
            const void *t = a.cur;
            a.cur = a.nxt;
            a.nxt = const_cast<void *>(t);
        }
        a.out = a.nxt;  // in place
        const int n = d.n0 + jj;
        a.step = n & 0x3fffffff;
        a.zdown = 0;
        a.trace_row = d.traces ? d.traces + (size_t)n * d.nrec : nullptr;
        a.src_ptr = d.src ? d.src + jj : nullptr;
        a.src_val = 0.f;
        if (!d.src)
            a.src_z = -1;
        tile_step<WAVE_F32, TXV, TY, RY, kFwd, true>(a, lid);
        // completion: every thread's stores have reached the L2 (the wait
        // covers stores on this architecture) before the counter moves
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(p.done + fs.done + lid, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One thread per interior cell, every tap read from global memory: a
// deliberately plain kernel used to cross-check the tiled one.  Same FP32
// operations in the same order, so the two agree bit for bit.
template <int KIND>
__global__ __launch_bounds__(256) void step_naive(StepArgs a)
{
    constexpr bool SCALED = Store<KIND>::scaled;
    Scales sc{1.f, 1.f, 1.f, 1.f, 0};
    Folded fd{a.c, 2.f, 1.f, 1.f};
    if constexpr (SCALED) {
        sc = step_scales<KIND>(a);
        publish_scale(a, sc, blockIdx.x, threadIdx.x);
        fd = fold_scales(a.c, sc, a.k_scale);
    }
    const Coefs &c = fd.c;
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float amax = 0.f;
    if (i < n) {
        const int x = (int)(i % a.nx);
        const int y = (int)((i / a.nx) % a.ny);
        const int z = (int)(i / ((long long)a.nx * a.ny));
        const long long p =
            (long long)(z + kGhost) * a.plane + (long long)(y + kGhost) * a.px + a.x0 + x;
        auto U = [&](long long q) { return read_elem<KIND>(a.cur, q, 1.f); };
        const float u = U(p);
        // same form and order as the tiled kernel (difference form for FP32)
        const float u2 = SCALED ? 0.f : 2.f * u;
        float lap = SCALED ? c.ctr * u : 0.f;
        for (int m = 1; m <= 4; ++m) {
            lap = fmaf(c.cx[m - 1], (U(p + m) + U(p - m)) - u2, lap);
            lap = fmaf(c.cy[m - 1], (U(p + (long long)m * a.px) + U(p - (long long)m * a.px)) - u2, lap);
            lap = fmaf(c.cz[m - 1], (U(p + m * a.plane) + U(p - m * a.plane)) - u2, lap);
        }
        const float g = a.gx[x] * a.gy[y] * a.gz[z];
        const float kk = read_elem<KIND>(a.k, p, 1.f);
        const float pp = read_elem<KIND>(Store<KIND>::uv ? a.dlt : a.nxt, p, 1.f);
        float t, pe;
        if constexpr (SCALED) {
            t = fmaf(kk, lap, fd.two_a * u);
            if constexpr (Store<KIND>::uv)
                pe = fmaf(-fd.b, pp, fd.a * u);
            else
                pe = fd.b * pp;
        } else {
            t = fmaf(kk, lap, 2.f * u);
            pe = pp;
        }
        t = fmaf(-g, pe, t);
        float v = g * t;
        if (z == a.src_z && y == a.src_y && x == a.src_x)
            v += src_value(a) * sc.out_inv;
        if constexpr (KIND == WAVE_F32) {
            static_cast<float *>(a.out)[p] = v;
        } else {
            static_cast<unsigned short *>(a.out)[p] = (unsigned short)Store<KIND>::enc(v);
            if constexpr (Store<KIND>::uv)
                static_cast<unsigned short *>(a.dlt)[p] =
                    (unsigned short)Store<KIND>::enc(0.5f * (v - fd.a * u));
            amax = fabsf(v);
        }
    }
    if constexpr (SCALED)
        fold_max(a, amax * sc.out);
}

// Receivers for the naive kernel (separate launch: it has no tile
// epilogue).  With 16-bit storage the scale of u^{n+1} is the one the step
// just published.
template <int KIND>
__global__ void sample_naive(const void *__restrict__ f, const long long *__restrict__ off, int nrec,
                             float *row, const int *exps, int slot)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrec) {
        const float scale = Store<KIND>::scaled ? ldexpf(1.f, exps[slot]) : 1.f;
        row[r] = read_elem<KIND>(f, off[r], scale);
    }
}


// Interior copy between two layouts with an exact power-of-two rescale:
// FP32 k into 16-bit storage (init), or a field of any storage into FP32
// (export).  `exps`/`slot` select a device exponent for the source scale.
template <int SRC, int DST>
__global__ __launch_bounds__(256) void convert_interior(const void *__restrict__ src, void *dst, int nx,
                                                        int ny, int nz, int spx, int sx0,
                                                        long long splane, int dpx, int dx0,
                                                        long long dplane, float scale,
                                                        const int *exps, int slot)
{
    const long long n = (long long)nx * ny * nz;
    const float sc = exps ? ldexpf(1.f, exps[slot]) : scale;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / ((long long)nx * ny));
        const long long si = (long long)(z + kGhost) * splane + (long long)(y + kGhost) * spx + sx0 + x;
        const long long di = (long long)(z + kGhost) * dplane + (long long)(y + kGhost) * dpx + dx0 + x;
        const float v = read_elem<SRC>(src, si, 1.f);
        if constexpr (DST == WAVE_F32)
            static_cast<float *>(dst)[di] = v * sc;
        else
            static_cast<unsigned short *>(dst)[di] = (unsigned short)Store<DST>::enc(v * sc);
    }
}

}  // namespace wavek
