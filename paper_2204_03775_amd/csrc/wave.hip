// libwave.so host side: contexts, launch planning, the checkpointed
// gradient driver, batched runs and the C ABI of include/wave.h.  The
// kernels live in wave_step.h (instantiated by the k_*.hip units).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "wave.h"
#include "wave_dev.h"
#include "wave_kernels.h"

using namespace wavek;

// Scratch of wave_check_noalloc: its two counters live in this fixed device
// array (one copy per GPU, kept until the process ends), so that the call
// allocates nothing.  On the host `scratch` is only a stand-in for the
// symbol, not a device address: host code uses the address
// hipGetSymbolAddress returns for each device (scratch_for), never the name.
constexpr int kScratchInts = 64;
static __device__ __align__(256) int scratch[kScratchInts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
int *scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (wave_init does it for the context's device).
int scratch_for(int device, int **out)
{
    if (device < 0 || device >= kMaxDevices)
        return WAVE_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess)
            return WAVE_EHIP;
        if (cur != device && hipSetDevice(device) != hipSuccess)
            return WAVE_EHIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device)
            (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return WAVE_EHIP;
        scratch_dev[device] = static_cast<int *>(p);
    }
    *out = scratch_dev[device];
    return WAVE_OK;
}

}  // namespace

namespace {
// ---------------------------------------------------------------------------
// host side

typedef void (*StepKernel)(StepArgs);
typedef void (*BatchKernel)(const ShotDesc *, BatchItems, int);
typedef void (*FlowKernel)(const ShotDesc *, FlowPlan);
typedef void (*RunKernel)(const ShotDesc *, BatchItems, RunSync);

struct Variant {
    const char *name;
    StepKernel fn[kNumKinds];  // by storage type; all NULL for "auto" and "naive"
    BatchKernel batch[3];      // FP32, FP16, BF16 (two-level storage)
    RunKernel run[3];          // the same, every step of a run in one launch
    StepKernel adj[3];  // adjoint step, imaging step, fused adjoint + imaging (FP32)
    FlowKernel flow;    // data-flow batched step (FP32)
    StepKernel fwd_cached;  // FP32 step with cache-resident load policies
    int txv, ty, ry;
};

#define TILED(TXV, TY, RY)                                                                        \
    {step_tiled<WAVE_F32, TXV, TY, RY>, step_tiled<WAVE_F16, TXV, TY, RY>,                        \
     step_tiled<WAVE_BF16, TXV, TY, RY>, step_tiled<WAVE_F16_UV, TXV, TY, RY>,                    \
     step_tiled<WAVE_BF16_UV, TXV, TY, RY>},                                                      \
    {step_batch<WAVE_F32, TXV, TY, RY>, step_batch<WAVE_F16, TXV, TY, RY>,                        \
     step_batch<WAVE_BF16, TXV, TY, RY>},                                                         \
    {step_batch_run<WAVE_F32, TXV, TY, RY>, step_batch_run<WAVE_F16, TXV, TY, RY>,                \
     step_batch_run<WAVE_BF16, TXV, TY, RY>},                                                     \
    {adjoint_tiled<kAdj, TXV, TY, RY>, adjoint_tiled<kImg, TXV, TY, RY>, adjoint_tiled<kFus, TXV, TY, RY>}, \
    step_flow<TXV, TY, RY>, step_tiled_cached<TXV, TY, RY>

const Variant kVariants[] = {
    {"auto", {nullptr, nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr},
     {nullptr, nullptr, nullptr}, nullptr, nullptr, 0, 0, 0},
    {"naive", {nullptr, nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr},
     {nullptr, nullptr, nullptr}, nullptr, nullptr, 0, 0, 0},
    {"t64x16_r1", TILED(16, 16, 1), 16, 16, 1},
    {"t128x8_r1", TILED(32, 8, 1), 32, 8, 1},
    {"t128x16_r2", TILED(32, 8, 2), 32, 8, 2},
    {"t64x32_r2", TILED(16, 16, 2), 16, 16, 2},
    {"t128x16_r1", TILED(32, 16, 1), 32, 16, 1},
    {"t256x8_r2", TILED(64, 4, 2), 64, 4, 2},
    {"t64x16_r2", TILED(16, 8, 2), 16, 8, 2},
    {"t128x32_r4", TILED(32, 8, 4), 32, 8, 4},
    {"t256x8_r1", TILED(64, 8, 1), 64, 8, 1},
    {"t64x32_r1", TILED(16, 32, 1), 16, 32, 1},
    {"t128x32_r2", TILED(32, 16, 2), 32, 16, 2},
    {"t256x16_r2", TILED(64, 8, 2), 64, 8, 2},
};
#undef TILED
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kNaive = 1;
const StepKernel kNaiveFn[kNumKinds] = {step_naive<WAVE_F32>, step_naive<WAVE_F16>, step_naive<WAVE_BF16>,
                                        step_naive<WAVE_F16_UV>, step_naive<WAVE_BF16_UV>};

// Whether the cells an FP32 step touches in its three fields (u^n, u^{n-1},
// k: the interior and 4 ghost rows and planes on each side) fit in the
// GPU's 256 MiB memory-side cache with room to spare.  Then every field
// keeps the default cache policy (step_tiled_cached): u^{n-1} and k, read
// once per step, are still cached when the next step reads them.  Measured
// with the step's access pattern: 13 % faster at 256^3 (about 210 MiB),
// 8-13 % slower at 384^3, where streaming them is better.
constexpr long long kCacheResidentBytes = 224ll << 20;
bool fits_in_cache(int nx, int ny, int nz)
{
    return 3ll * 4 * (nx + 8) * (ny + 8) * (long long)(nz + 8) <= kCacheResidentBytes;
}

// The element encoding of a storage type (the u-and-change types store
// both of their fields in the encoding of their base type).
int base_kind(int kind) { return kind == WAVE_F16_UV ? WAVE_F16 : kind == WAVE_BF16_UV ? WAVE_BF16 : kind; }

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Launch geometry of a tiled (or the naive) kernel over one grid.
struct Geo {
    int v = 0, ntx = 0, nty = 0, nchunks = 0, zc = 0, nwg = 0, grid = 0;
};

}  // namespace

// State of the gradient computation (FP32 storage): the checkpoints and the
// level store of the last checkpointed forward run, the adjoint fields and
// the FP64 accumulator, all in the field layout (ghost cells zero).
struct wave_grad_state {
    int64_t step0 = 0;  // step counter at the start of the forward run
    int nt = 0;         // steps of the run (0: no run recorded)
    int every = 0;      // segment length C
    int nseg = 0;       // segments: segment i covers steps i*C .. min((i+1)*C, nt) - 1
    int held = -1;      // segment whose levels c+1 .. the store holds
    bool has_src = false;
    void *slab = nullptr;  // 2 * nseg checkpoint levels, then C store levels
    size_t slab_levels = 0;
    float *src = nullptr;  // the run's source values [nt]
    int src_cap = 0;
    void *phi[2] = {nullptr, nullptr};
    double *acc = nullptr;
    // receiver cells (distinct) and, per cell, its receivers
    long long *cell_off = nullptr;
    int *cell_start = nullptr, *cell_rec = nullptr;
    int ncells = -1;
    std::vector<long long> cell_off_host;  // the cells' offsets, host copy
};

struct wave_ctx {
    wave_params_t p;
    wave_layout_t lay;    // layout of the u fields (and of the stored k)
    wave_layout_t lay32;  // FP32 layout (the caller's k for 16-bit storage)
    int device = 0;
    hipStream_t stream = nullptr;
    const void *k = nullptr;  // stored k: the caller's (FP32) or k16
    void *k16 = nullptr;      // library-owned 16-bit k
    float k_scale = 1.f;
    void *buf0 = nullptr, *buf1 = nullptr;  // roles at init: cur, prev
    void *dbuf = nullptr;                   // d^n (u-and-change storage), library-owned
    void *cur = nullptr, *prev = nullptr;
    int64_t step = 0;
    unsigned zflip = 0;  // tiled launches so far: their z-march directions alternate
    bool cache_resident = false;  // FP32 fields small enough to stay in the memory-side cache
    int src[3] = {-1, -1, -1};
    std::vector<int32_t> rec;  // [nrec][3]
    int nrec = 0;
    float *traces = nullptr;
    int32_t trace_cap = 0;
    Coefs coefs{};
    // device tables
    float *gx = nullptr, *gy = nullptr, *gz = nullptr;
    long long *rec_off_all = nullptr;  // receiver offsets in receiver order (naive sampling)
    int *rec_start = nullptr;
    long long *rec_off = nullptr;
    int *rec_idx = nullptr;
    int *ring = nullptr;  // [8]: exps[4] then maxes[4] (16-bit storage)
    // launch configuration
    int variant = 0, zchunk = 0;  // requested (0 = auto)
    int v_used = 0, zc_used = 0;
    int ntx = 0, nty = 0, nchunks = 0, nwg = 0, grid = 0;
    wave_grad_state g;
    bool fuse_adjoint = true;  // adjoint step and imaging term in one pass
    // graph replay of wave_run: the launches of the last captured run and
    // the state it started from
    struct RunGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int64_t step0 = -1;
        int nsteps = 0;
        const float *src = nullptr;
        float *traces = nullptr;
        void *cur = nullptr, *prev = nullptr;
    } rg;
    bool use_graph = false;
    std::string err;
};

namespace {

int fail(wave_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), WAVE_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

void sponge_profile(int n, int width, double alpha, std::vector<float> &g)
{
    g.assign(n, 1.0f);
    for (int i = 0; i < n; ++i) {
        const int d = std::min(i, n - 1 - i);
        if (d < width) {
            const double t = alpha * double(width - d);
            g[i] = float(std::exp(-t * t));
        }
    }
}

// Choose a variant and z-chunk; fill the grid geometry.  Measured on the
// 512^3 workload:
//   - FP32: 512-thread work-groups with one float4 per thread, about one
//     per CU (z split into as many chunks as that takes), beat both smaller
//     work-groups and more of them; 256 x 8 tiles edge out 128 x 16 and
//     64 x 32 by about 1.5%;
//   - 16-bit storage moves half the bytes per load, so a thread needs two
//     rows to keep enough bytes in flight: 128 x 32 tiles of two rows per
//     thread at 256 work-groups run 594 Gpts/s against 482 for 256 x 8;
//   - u-and-change storage (five streams) does best with 128 x 16 tiles of
//     two rows per thread at 512 work-groups (478 against 361);
//   - in every case the best z split fills whole rounds of the work-groups
//     the GPU holds at once (one or two per CU here): 755 x 994 tiles of
//     256 x 8 in one chunk are 375 work-groups, a round and a half of 256.
// Every chunk re-reads 8 planes of u^n, so chunks are kept at >= 32 planes.
// Grids of fewer than 2^22 cells fit in the caches and are latency-bound:
// there, about 512 work-groups with chunks down to one plane run 3-6x
// faster per step than 32-plane chunks (48^3: 3.9 against 24.8 us per
// step; 128^3: 9.5 against 25.9; 192^3: about 25 against 29).
constexpr int kAutoVariant = 10;     // t256x8_r1 (FP32)
constexpr int kAutoNarrowVariant = 6;  // t128x16_r1 (FP32 when 256-wide tiles would idle lanes)
constexpr int kAuto16Variant = 4;    // t128x16_r2 (FP16 / BF16, two levels)
constexpr int kAutoUvVariant = 12;   // t128x32_r2 (u-and-change storage)
constexpr int kSmallVariant = 2;     // t64x16_r1 for grids of fewer than 2^22 cells
constexpr int kTargetWorkgroupsSmall = 512;
constexpr int kMinChunk = 32;
constexpr int kMinChunkSmall = 1;
constexpr int kMinChunkNarrow = 8;

// Work-groups of the tiled kernel of variant v that the current GPU holds at
// once (occupancy per CU times CUs).
// Work-groups of variant v that make one round: 8 waves (512 threads) per
// CU, as one work-group of 512 threads or two of 256, bounded by how many
// fit at once (occupancy API).  Two resident 512-thread work-groups per CU
// measured slower than one: they split the CU's bandwidth and add a tail.
long long round_workgroups(int kind, int v)
{
    const Variant &V = kVariants[v];
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const StepKernel f = kind == WAVE_F32 || V.fn[kind] ? V.fn[kind] : V.fn[WAVE_F32];
    const int threads = V.txv * V.ty;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return (long long)cus * std::min(per_cu, std::max(1, 512 / threads));
}

// z-chunk length for a grid of `tiles` x-y tiles and rounds of `cap`
// work-groups: the chunk count that maximises
//     nwg / (R cap) * 0.85^(R-1) / (1 + 2/zc),   R = ceil(nwg / cap)
// (the maximum is stored in *score when score is not null).
// The step time follows the rounds the busiest CU runs, so work-group counts
// just under a multiple of a round are the efficient ones; each further
// round costs about 15 % beyond its share (idle time at the hand-over), and
// each chunk re-reads 8 planes of u^n (a quarter of the bytes per update:
// factor 1 + 2/zc).  Chunks stay >= min_chunk planes (or nz).  Fitted on
// 16 grids from 112 x 304 x 240 to 600 x 1200 x 200, every chunk count
// measured, with 128 x 16 tiles; the other large-grid plans it gives are
// the ones measured best before it.
int fill_rounds_chunk(long long tiles, int nz, int min_chunk, long long cap, double *score = nullptr)
{
    double best = -1.0;
    int zc = nz;
    for (int c = 1; c <= nz; ++c) {
        const int z = (nz + c - 1) / c;
        if (z < std::min(min_chunk, nz))
            break;
        if (c > 1 && z == (nz + c - 2) / (c - 1))
            continue;  // the same chunk length as c - 1
        const long long nwg = tiles * ((nz + z - 1) / z);
        const long long rounds = (nwg + cap - 1) / cap;
        const double eff = double(nwg) / double(rounds * cap) * std::pow(0.85, double(rounds - 1)) /
                           (1.0 + 2.0 / z);
        if (eff > best + 1e-12) {
            best = eff;
            zc = z;
        }
    }
    if (score)
        *score = best;
    return zc;
}

// How well tiles of tx x tyr cells fit an nx x ny plane, for a bandwidth-
// bound step: the share of x lanes inside the grid, times how even the
// tiles' work is (mean over tiles / the largest).  A plane one tile wide has
// idle lanes but equal tiles; a plane with a thin last tile column leaves
// the CUs that run that column idle at the end of the round.
double tile_fit(int nx, int ny, int tx, int tyr)
{
    const int ntx = (nx + tx - 1) / tx, nty = (ny + tyr - 1) / tyr;
    const double lanes = double(nx) / (double(ntx) * tx);
    const double even = (double(nx) / ntx) / std::min(tx, nx) * ((double(ny) / nty) / std::min(tyr, ny));
    return lanes * even;
}

Geo plan_geo(int nx, int ny, int nz, int kind, int variant, int zchunk)
{
    Geo g;
    int v = variant;
    const bool large = (long long)nx * ny * nz >= (1ll << 22);
    // FP32 grids whose x extent leaves more than 5 % of a 256-wide tile's
    // lanes idle ("narrow") choose between 128 x 16 and 256 x 8 tiles by
    // fit times the chunk rule's round efficiency (128 x 16 on a tie)
    const bool narrow = large && kind == WAVE_F32 && variant == 0 &&
                        double(nx) / (256.0 * ((nx + 255) / 256)) < 0.95;
    if (narrow && zchunk <= 0) {
        double best = -1.0;
        for (const int cand : {kAutoNarrowVariant, kAutoVariant}) {
            const Variant &C = kVariants[cand];
            const int tx = 4 * C.txv, tyr = C.ty * C.ry;
            const long long tiles = (long long)((nx + tx - 1) / tx) * ((ny + tyr - 1) / tyr);
            double eff = 0.0;
            (void)fill_rounds_chunk(tiles, nz, kMinChunkNarrow, round_workgroups(kind, cand), &eff);
            eff *= tile_fit(nx, ny, tx, tyr);
            if (eff > best * (1.0 + 1e-9)) {
                best = eff;
                v = cand;
            }
        }
    }
    if (v == 0)
        v = !large ? kSmallVariant
                   : kind == WAVE_F32 ? (narrow ? kAutoNarrowVariant : kAutoVariant)
                                      : is_uv(kind) ? kAutoUvVariant : kAuto16Variant;
    g.v = v;
    if (v == kNaive) {
        g.ntx = g.nty = g.nchunks = 0;
        g.zc = nz;
        long long n = (long long)nx * ny * nz;
        g.nwg = g.grid = int((n + 255) / 256);
        return g;
    }
    const Variant &V = kVariants[v];
    const int tx = 4 * V.txv, tyr = V.ty * V.ry;
    g.ntx = (nx + tx - 1) / tx;
    g.nty = (ny + tyr - 1) / tyr;
    const long long tiles = (long long)g.ntx * g.nty;
    int zc = zchunk;
    if (zc <= 0 && !large) {
        const long long chunks = std::max(1ll, (kTargetWorkgroupsSmall + tiles / 2) / tiles);
        zc = std::max(int((nz + chunks - 1) / chunks), std::min(kMinChunkSmall, nz));
    } else if (zc <= 0) {
        // large grids: whole rounds, chunks of at least 32 planes (8 for
        // the narrow-grid tiles, whose tiles are few)
        zc = fill_rounds_chunk(tiles, nz, narrow ? kMinChunkNarrow : kMinChunk, round_workgroups(kind, v));
    }
    if (zc > nz)
        zc = nz;
    g.zc = zc;
    g.nchunks = (nz + zc - 1) / zc;
    g.nwg = int(tiles * g.nchunks);
    g.grid = int(round_up(g.nwg, 8));
    return g;
}

void plan_launch(wave_ctx *c)
{
    const Geo g = plan_geo(c->p.nx, c->p.ny, c->p.nz, c->p.dtype, c->variant, c->zchunk);
    c->v_used = g.v;
    c->ntx = g.ntx;
    c->nty = g.nty;
    c->nchunks = g.nchunks;
    c->zc_used = g.zc;
    c->nwg = g.nwg;
    c->grid = g.grid;
}

long long elem_offset(const wave_layout_t &l, int z, int y, int x)
{
    return ((long long)(z + kGhost) * l.rows + (y + kGhost)) * l.pitch_x + l.x_offset + x;
}

template <class T>
void free_dev(T *&p)
{
    if (p) {
        (void)hipFree(p);
        p = nullptr;
    }
}

// Per-work-group receiver lists for the tiled kernels.
int build_receiver_tables(wave_ctx *c)
{
    free_dev(c->rec_start);
    free_dev(c->rec_off);
    free_dev(c->rec_idx);
    if (c->v_used == kNaive)
        return WAVE_OK;
    const Variant &V = kVariants[c->v_used];
    const int tx = 4 * V.txv, tyr = V.ty * V.ry;
    std::vector<int> start(c->nwg + 1, 0), owner(c->nrec);
    for (int r = 0; r < c->nrec; ++r) {
        const int z = c->rec[3 * r], y = c->rec[3 * r + 1], x = c->rec[3 * r + 2];
        const int lid = ((z / c->zc_used) * c->nty + y / tyr) * c->ntx + x / tx;
        owner[r] = lid;
        start[lid + 1]++;
    }
    for (int i = 0; i < c->nwg; ++i)
        start[i + 1] += start[i];
    std::vector<int> fill(start.begin(), start.end() - 1), idx(std::max(c->nrec, 1));
    std::vector<long long> off(std::max(c->nrec, 1));
    for (int r = 0; r < c->nrec; ++r) {
        const int slot = fill[owner[r]]++;
        idx[slot] = r;
        off[slot] = elem_offset(c->lay, c->rec[3 * r], c->rec[3 * r + 1], c->rec[3 * r + 2]);
    }
    HIP_TRY(c, hipMalloc(&c->rec_start, sizeof(int) * start.size()));
    HIP_TRY(c, hipMalloc(&c->rec_off, sizeof(long long) * off.size()));
    HIP_TRY(c, hipMalloc(&c->rec_idx, sizeof(int) * idx.size()));
    HIP_TRY(c, hipMemcpy(c->rec_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->rec_off, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->rec_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
    return WAVE_OK;
}

StepArgs make_args(const wave_ctx *c)
{
    StepArgs a;
    a.k = c->k;
    a.cur = c->cur;
    a.nxt = c->prev;
    a.gx = c->gx;
    a.gy = c->gy;
    a.gz = c->gz;
    a.c = c->coefs;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.px = int(c->lay.pitch_x);
    a.x0 = int(c->lay.x_offset);
    a.plane = c->lay.plane;
    a.nxq = (c->p.nx + 3) / 4;
    a.ntx = c->ntx;
    a.nty = c->nty;
    a.nchunks = c->nchunks;
    a.zc = c->zc_used;
    a.nwg = c->nwg;
    a.src_z = c->src[0];
    a.src_y = c->src[1];
    a.src_x = c->src[2];
    a.src_ptr = nullptr;
    a.src_val = 0.f;
    a.rec_start = c->rec_start;
    a.rec_off = c->rec_off;
    a.rec_idx = c->rec_idx;
    a.trace_row = (c->traces && c->nrec > 0) ? c->traces + (size_t)c->step * c->nrec : nullptr;
    a.step = int(c->step & 0x3fffffff);
    a.k_scale = c->k_scale;
    a.exps = c->ring;
    a.maxes = reinterpret_cast<unsigned *>(c->ring + 4);
    a.out = c->prev;
    a.grad = nullptr;
    a.aux = nullptr;
    a.dlt = c->dbuf;
    a.zdown = 0;
    return a;
}

// One forward step from (cur = u^n, prev = u^{n-1}) into `out` (== prev for
// the in-place step), step counter and trace row as given.
int enqueue_forward(wave_ctx *c, void *cur, void *prev, void *out, const float *src_ptr, float src_val,
                    int64_t step, float *trace_row)
{
    StepArgs a = make_args(c);
    a.cur = cur;
    a.nxt = prev;
    a.out = out;
    a.src_ptr = src_ptr;
    a.src_val = src_val;
    a.step = int(step & 0x3fffffff);
    a.trace_row = trace_row;
    a.zdown = int(c->zflip++ & 1u);

    const int kind = c->p.dtype;
    if (c->v_used == kNaive) {
        hipLaunchKernelGGL(kNaiveFn[kind], dim3(c->grid), dim3(256), 0, c->stream, a);
        if (a.trace_row) {
            const dim3 g((c->nrec + 255) / 256), b(256);
            const int slot = (a.step + 1) & 3;
            const void *f = out;
            const long long *off = c->rec_off_all;
            const int *ex = c->ring;
            const int bk = base_kind(kind);
            if (bk == WAVE_F32)
                hipLaunchKernelGGL(sample_naive<WAVE_F32>, g, b, 0, c->stream, f, off, c->nrec,
                                   a.trace_row, ex, slot);
            else if (bk == WAVE_F16)
                hipLaunchKernelGGL(sample_naive<WAVE_F16>, g, b, 0, c->stream, f, off, c->nrec,
                                   a.trace_row, ex, slot);
            else
                hipLaunchKernelGGL(sample_naive<WAVE_BF16>, g, b, 0, c->stream, f, off, c->nrec,
                                   a.trace_row, ex, slot);
        }
    } else {
        const Variant &V = kVariants[c->v_used];
        const StepKernel fn = (c->cache_resident && V.fwd_cached) ? V.fwd_cached : V.fn[kind];
        hipLaunchKernelGGL(fn, dim3(c->grid), dim3(V.txv * V.ty), 0, c->stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(c, WAVE_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return WAVE_OK;
}

float *trace_row_of(const wave_ctx *c, int64_t step)
{
    return (c->traces && c->nrec > 0) ? c->traces + (size_t)step * c->nrec : nullptr;
}

int launch_step(wave_ctx *c, const float *src_ptr, float src_val)
{
    const int rc = enqueue_forward(c, c->cur, c->prev, c->prev, src_ptr, src_val, c->step,
                                   trace_row_of(c, c->step));
    if (rc != WAVE_OK)
        return rc;
    // u^{n+1} now lives in the old u^{n-1} buffer
    void *t = c->prev;
    c->prev = c->cur;
    c->cur = t;
    c->step += 1;
    return WAVE_OK;
}

int check_trace_room(wave_ctx *c, int64_t nsteps)
{
    if (c->traces && c->nrec > 0 && c->step + nsteps > c->trace_cap)
        return fail(c, WAVE_EINVAL, "trace buffer holds %d rows; steps %lld..%lld requested",
                    c->trace_cap, (long long)c->step, (long long)(c->step + nsteps - 1));
    return WAVE_OK;
}

void free_grad(wave_grad_state &g)
{
    free_dev(g.slab);
    free_dev(g.src);
    free_dev(g.phi[0]);
    free_dev(g.phi[1]);
    free_dev(g.acc);
    free_dev(g.cell_off);
    free_dev(g.cell_start);
    free_dev(g.cell_rec);
    g = wave_grad_state();
}

void drop_run_graph(wave_ctx *c)
{
    if (c->rg.exec) {
        (void)hipStreamSynchronize(c->stream);  // it may still be running
        (void)hipGraphExecDestroy(c->rg.exec);
    }
    if (c->rg.graph)
        (void)hipGraphDestroy(c->rg.graph);
    c->rg = wave_ctx::RunGraph();
}

void free_device(wave_ctx *c)
{
    drop_run_graph(c);
    free_grad(c->g);
    free_dev(c->gx);
    free_dev(c->gy);
    free_dev(c->gz);
    free_dev(c->rec_off_all);
    free_dev(c->rec_start);
    free_dev(c->rec_off);
    free_dev(c->rec_idx);
    free_dev(c->ring);
    free_dev(c->k16);
    free_dev(c->dbuf);
}

int launch_convert(hipStream_t s, int src_kind, int dst_kind, const void *src, void *dst, int nx, int ny,
                   int nz, const wave_layout_t &sl, const wave_layout_t &dl, float scale,
                   const int *exps, int slot)
{
    src_kind = base_kind(src_kind);
    dst_kind = base_kind(dst_kind);
    const long long n = (long long)nx * ny * nz;
    const dim3 g((unsigned)std::min<long long>((n + 255) / 256, 8192)), b(256);
    const int spx = int(sl.pitch_x), sx0 = int(sl.x_offset), dpx = int(dl.pitch_x),
              dx0 = int(dl.x_offset);
    const long long sp = sl.plane, dp = dl.plane;
#define CONV(S, D)                                                                                 \
    hipLaunchKernelGGL((convert_interior<S, D>), g, b, 0, s, src, dst, nx, ny, nz, spx, sx0, sp, dpx, \
                       dx0, dp, scale, exps, slot)
    if (src_kind == WAVE_F32 && dst_kind == WAVE_F16)
        CONV(WAVE_F32, WAVE_F16);
    else if (src_kind == WAVE_F32 && dst_kind == WAVE_BF16)
        CONV(WAVE_F32, WAVE_BF16);
    else if (src_kind == WAVE_F16 && dst_kind == WAVE_F32)
        CONV(WAVE_F16, WAVE_F32);
    else if (src_kind == WAVE_BF16 && dst_kind == WAVE_F32)
        CONV(WAVE_BF16, WAVE_F32);
    else if (src_kind == WAVE_F32 && dst_kind == WAVE_F32)
        CONV(WAVE_F32, WAVE_F32);
    else
        return WAVE_EINVAL;
#undef CONV
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

// ---------------------------------------------------------------------------
// gradient with respect to k: checkpointed forward run, adjoint run

Geo ctx_geo(const wave_ctx *c)
{
    Geo g;
    g.v = c->v_used;
    g.ntx = c->ntx;
    g.nty = c->nty;
    g.nchunks = c->nchunks;
    g.zc = c->zc_used;
    g.nwg = c->nwg;
    g.grid = c->grid;
    return g;
}

// The adjoint and imaging steps use the context's tiling when one was
// configured, else their own automatic choice: the fused pass holds two
// stencil fields, and at 256 x 8 tiles it needs more than the 256 registers
// two waves per SIMD allow (it spills), while 128 x 16 tiles fit (241).
constexpr int kAdjointAutoVariant = 6;  // t128x16_r1 for grids of >= 2^22 cells

Geo adjoint_geo(const wave_ctx *c)
{
    if (c->variant != 0 && c->v_used != kNaive)
        return ctx_geo(c);
    const long long pts = (long long)c->p.nx * c->p.ny * c->p.nz;
    return plan_geo(c->p.nx, c->p.ny, c->p.nz, WAVE_F32, pts >= (1ll << 22) ? kAdjointAutoVariant : kSmallVariant,
                    0);
}

int enqueue_adjoint(wave_ctx *c, const Geo &geo, int mode, const void *cur, void *nxt, void *out,
                    double *acc, const void *aux = nullptr)
{
    StepArgs a = make_args(c);
    a.cur = cur;
    a.nxt = nxt;
    a.out = out;
    a.grad = acc;
    a.aux = aux;
    a.ntx = geo.ntx;
    a.nty = geo.nty;
    a.nchunks = geo.nchunks;
    a.zc = geo.zc;
    a.nwg = geo.nwg;
    a.src_z = a.src_y = a.src_x = -1;
    a.src_ptr = nullptr;
    a.trace_row = nullptr;
    a.zdown = int(c->zflip++ & 1u);
    const Variant &V = kVariants[geo.v];
    hipLaunchKernelGGL(V.adj[mode - 1], dim3(geo.grid), dim3(V.txv * V.ty), 0, c->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(c, WAVE_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
    return WAVE_OK;
}

size_t level_bytes(const wave_ctx *c) { return (size_t)c->lay.bytes; }

// Level l of segment `seg`: a^{c-1} and a^c from the checkpoint, a^{c+1} ..
// a^{c+C} from the store (c = seg * C).
void *level_ptr(wave_ctx *c, int seg, int64_t l)
{
    wave_grad_state &g = c->g;
    const int64_t c0 = (int64_t)seg * g.every;
    char *base = static_cast<char *>(g.slab);
    const size_t lb = level_bytes(c);
    if (l <= c0)
        return base + lb * (size_t)(2 * seg + (l == c0 ? 1 : 0));
    return base + lb * (size_t)(2 * g.nseg + (l - c0 - 1));
}

// Out-of-place forward steps of segment `seg` from its checkpoint, writing
// levels c+1 .. c+count into the store; traces are written when `record`.
int forward_segment(wave_ctx *c, int seg, int count, bool record)
{
    wave_grad_state &g = c->g;
    const int64_t c0 = (int64_t)seg * g.every;
    for (int j = 0; j < count; ++j) {
        const int64_t n = c0 + j;  // this step writes a^{n+1}
        const float *sp = g.has_src ? g.src + n : nullptr;
        const int rc = enqueue_forward(c, level_ptr(c, seg, n), level_ptr(c, seg, n - 1),
                                       level_ptr(c, seg, n + 1), sp, 0.f, g.step0 + n,
                                       record ? trace_row_of(c, g.step0 + n) : nullptr);
        if (rc != WAVE_OK)
            return rc;
    }
    g.held = seg;
    return WAVE_OK;
}

// Distinct receiver cells with their receivers (the adjoint source adds the
// trace derivatives of every receiver at a cell).
int build_receiver_cells(wave_ctx *c)
{
    wave_grad_state &g = c->g;
    if (g.ncells >= 0)
        return WAVE_OK;
    std::vector<std::pair<long long, int>> r(c->nrec);
    for (int i = 0; i < c->nrec; ++i)
        r[i] = {elem_offset(c->lay, c->rec[3 * i], c->rec[3 * i + 1], c->rec[3 * i + 2]), i};
    std::sort(r.begin(), r.end());
    std::vector<long long> off;
    std::vector<int> start, idx;
    for (int i = 0; i < c->nrec; ++i) {
        if (i == 0 || r[i].first != r[i - 1].first) {
            off.push_back(r[i].first);
            start.push_back(i);
        }
        idx.push_back(r[i].second);
    }
    start.push_back(c->nrec);
    g.ncells = int(off.size());
    g.cell_off_host = off;
    off.resize(std::max<size_t>(off.size(), 1));
    idx.resize(std::max<size_t>(idx.size(), 1));
    HIP_TRY(c, hipMalloc(&g.cell_off, sizeof(long long) * off.size()));
    HIP_TRY(c, hipMalloc(&g.cell_start, sizeof(int) * start.size()));
    HIP_TRY(c, hipMalloc(&g.cell_rec, sizeof(int) * idx.size()));
    HIP_TRY(c, hipMemcpy(g.cell_off, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(g.cell_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(g.cell_rec, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
    return WAVE_OK;
}

// Segment length when the caller leaves it to the library: every level of
// the run when that fits in half of the free device memory, else the
// largest C whose checkpoints and store (2 ceil(nt / C) + C levels) fit.
int auto_segment(const wave_ctx *c, int nt)
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
        return -1;
    const double budget = 0.5 * double(free_b) / double(level_bytes(c));
    for (int C = nt; C >= 1; --C)
        if (2.0 * ((nt + C - 1) / C) + C <= budget)
            return C;
    return -1;
}

}  // namespace

// schedule 3's barrier words after a group's tickets: count, gen, abort, spare
constexpr int kRunSyncInts = 4;

struct wave_batch {
    struct Group {
        int kind = 0, variant = 0;
        std::vector<int> shots;       // indices into ctx
        std::vector<ShotDesc> h_desc; // last uploaded descriptors
        ShotDesc *d_desc = nullptr;
        int *d_items = nullptr;       // shot[items], lid[items], xcd_start[9], counters[16], run sync[4]
        BatchItems items{};
        int total = 0, grid = 0, threads = 0;
        // schedule 2: FlowShot table, xcd_shot[9], xcd_items[8], then the
        // counters cleared before every launch: tickets[8], done[], abort[1]
        int *d_flow = nullptr;
        FlowPlan plan{};
        int *flow_counters = nullptr;
        long long flow_ncounters = 0;
        int flow_grid = 0, flow_max_items = 0;
        // schedule 3: work-groups of the single-launch run (all resident)
        int run_grid = 0;
    };
    std::vector<wave_ctx *> ctx;
    std::vector<int> cfg;  // (variant, zchunk, nwg) of every shot at creation
    std::vector<Group> groups;
    hipStream_t stream = nullptr;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = -1;
    // schedule 1: every shot launched with its own configuration, shots
    // dealt to these streams (fork and join through events)
    int schedule = 0;
    int wait_limit = 1 << 24;  // schedule 2: polls before a dependency wait gives up
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> ev;  // fork, then one join per stream
    // schedule 1 under graph replay: one graph per stream, each replayed on
    // its own stream (one graph spanning the streams ran its branches one
    // after another, 1.15x slower than the same launches made eagerly)
    std::vector<hipGraph_t> sgraph;
    std::vector<hipGraphExec_t> sexec;
    std::vector<int64_t> key;    // the run the graph was captured for
    long long points = 0, workgroups = 0;
    std::string err;
};

namespace {

int bfail(wave_batch *b, int code, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return code;
}

void drop_batch_graph(wave_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (hipGraphExec_t e : b->sexec)
        if (e)
            (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : b->sgraph)
        if (g)
            (void)hipGraphDestroy(g);
    b->sexec.clear();
    b->sgraph.clear();
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = -1;
    b->key.clear();
}

void drop_streams(wave_batch *b)
{
    for (hipStream_t s : b->aux)
        (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->ev)
        (void)hipEventDestroy(e);
    b->aux.clear();
    b->ev.clear();
}

void drop_flow(wave_batch *b)
{
    for (auto &g : b->groups) {
        free_dev(g.d_flow);
        g.d_flow = nullptr;
        g.flow_counters = nullptr;
        g.flow_ncounters = 0;
    }
}

void batch_free(wave_batch *b)
{
    drop_batch_graph(b);
    drop_streams(b);
    drop_flow(b);
    for (auto &g : b->groups) {
        free_dev(g.d_desc);
        free_dev(g.d_items);
    }
}

// Schedule 2 is switched off: its first run on the GPU did not complete
// (no fault; the run exceeded its time limit), and neither a CPU replay of
// its ticket and dependency logic nor a check of the block-to-XCD mapping
// found the cause.  set_schedule rejects it until one is found.
constexpr bool kFlowScheduleEnabled = false;

// Schedule 2 plans: shots dealt to the 8 XCDs, largest first to the least
// loaded (in cells); per XCD the shots' items of one step, shot by shot.
int build_flow(wave_batch *b)
{
    int device = 0, cus = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        return WAVE_EHIP;
    for (auto &g : b->groups) {
        const Variant &V = kVariants[g.variant];
        const int ns = int(g.shots.size());
        std::vector<int> order(ns), xcd(ns);
        std::vector<double> cells(ns);
        for (int t = 0; t < ns; ++t) {
            const wave_ctx *c = b->ctx[g.shots[t]];
            order[t] = t;
            cells[t] = double(c->p.nx) * c->p.ny * c->p.nz;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cells[x] > cells[y]; });
        double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (const int t : order) {
            const int x = int(std::min_element(load, load + 8) - load);
            load[x] += cells[t];
            xcd[t] = x;
        }
        std::vector<FlowShot> fs;
        std::vector<int> xcd_shot(9, 0), xcd_items(8, 0);
        int done = 0;
        for (int x = 0; x < 8; ++x) {
            xcd_shot[x] = int(fs.size());
            for (const int t : order) {
                if (xcd[t] != x)
                    continue;
                const wave_ctx *c = b->ctx[g.shots[t]];
                FlowShot f{};
                f.desc = t;
                f.ntx = c->ntx;
                f.nty = c->nty;
                f.nch = (c->p.nz + c->zc_used - 1) / c->zc_used;
                f.items = f.ntx * f.nty * f.nch;
                f.base = xcd_items[x];
                f.done = done;
                f.zreach = (kGhost + c->zc_used - 1) / c->zc_used;
                xcd_items[x] += f.items;
                done += f.items;
                fs.push_back(f);
            }
        }
        xcd_shot[8] = int(fs.size());
        // blob: FlowShot table (as ints), xcd_shot, xcd_items, tickets, done, abort
        static_assert(sizeof(FlowShot) % sizeof(int) == 0, "FlowShot is a whole number of ints");
        const size_t nfs = fs.size() * (sizeof(FlowShot) / sizeof(int));
        const long long ncounters = 8 + (long long)done + 1;
        const size_t nints = nfs + 9 + 8 + size_t(ncounters);
        free_dev(g.d_flow);
        g.d_flow = nullptr;
        if (hipMalloc(&g.d_flow, sizeof(int) * nints) != hipSuccess)
            return WAVE_ENOMEM;
        std::vector<int> blob(nfs + 17, 0);
        std::memcpy(blob.data(), fs.data(), sizeof(FlowShot) * fs.size());
        std::copy(xcd_shot.begin(), xcd_shot.end(), blob.begin() + nfs);
        std::copy(xcd_items.begin(), xcd_items.end(), blob.begin() + nfs + 9);
        if (hipMemcpy(g.d_flow, blob.data(), sizeof(int) * blob.size(), hipMemcpyHostToDevice) != hipSuccess)
            return WAVE_EHIP;
        g.plan.shots = reinterpret_cast<const FlowShot *>(g.d_flow);
        g.plan.xcd_shot = g.d_flow + nfs;
        g.plan.xcd_items = g.d_flow + nfs + 9;
        g.flow_counters = g.d_flow + nfs + 17;
        g.flow_ncounters = ncounters;
        g.plan.tickets = g.flow_counters;
        g.plan.done = g.flow_counters + 8;
        g.plan.abort = g.flow_counters + 8 + done;
        g.flow_max_items = *std::max_element(xcd_items.begin(), xcd_items.end());
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V.flow, g.threads, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        g.flow_grid = int(round_up((long long)per_cu * cus, 8));
    }
    return WAVE_OK;
}

// Schedule 2: per group, launches of as many steps as the 32-bit tickets
// allow (normally the whole run), each after clearing its counters.
int flow_enqueue(wave_batch *b, int nsteps)
{
    for (auto &g : b->groups) {
        const long long cap = ((1ll << 31) - 1 - g.flow_grid) / std::max(1, g.flow_max_items);
        const int seg = int(std::max(1ll, std::min<long long>(cap, nsteps)));
        for (int j0 = 0; j0 < nsteps; j0 += seg) {
            FlowPlan p = g.plan;
            p.nsteps = std::min(seg, nsteps - j0);
            p.j0 = j0;
            p.wait_limit = b->wait_limit;
            const int zb = int(std::min<long long>((g.flow_ncounters + 255) / 256, 1024));
            hipLaunchKernelGGL(zero_ints, dim3(zb), dim3(256), 0, b->stream, g.flow_counters, g.flow_ncounters);
            hipLaunchKernelGGL(kVariants[g.variant].flow, dim3(g.flow_grid), dim3(g.threads), 0, b->stream,
                               (const ShotDesc *)g.d_desc, p);
        }
    }
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

// Schedule 3 plans: per group, as many work-groups as the GPU holds at once
// (the single-launch run waits at grid barriers, so all must be resident),
// a multiple of 8 so that every XCD's item range has its own work-groups.
int build_run(wave_batch *b)
{
    int device = 0, cus = 0, coop = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1 ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess)
        return WAVE_EHIP;
    if (!coop)
        return WAVE_EINVAL;
    for (auto &g : b->groups) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kVariants[g.variant].run[g.kind], g.threads, 0) !=
                hipSuccess ||
            per_cu < 1)
            return WAVE_EHIP;
        g.run_grid = int((long long)per_cu * cus / 8 * 8);
        if (g.run_grid < 8)
            return WAVE_EHIP;
    }
    return WAVE_OK;
}

// Schedule 3: per group, one cooperative launch for all nsteps steps, after
// clearing its tickets and barrier words.  Every barrier wait of the launch
// gives up (and flags the run as failed) past a wall-clock limit of 2 s plus
// 0.1 ms per step and 0.1 ns per cell-update (10 Gpts/s, far below the
// kernels' rates).
int run_enqueue(wave_batch *b, int nsteps)
{
    int device = 0, khz = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz < 1)
        return WAVE_EHIP;
    for (auto &g : b->groups) {
        long long cells = 0;
        for (int t : g.shots)
            cells += (long long)b->ctx[t]->p.nx * b->ctx[t]->p.ny * b->ctx[t]->p.nz;
        const double seconds = 2.0 + nsteps * (1e-4 + double(cells) * 1e-10);
        int *words = g.items.counters;
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(256), 0, b->stream, words, (long long)(16 + kRunSyncInts));
        RunSync rs;
        rs.count = reinterpret_cast<unsigned *>(words + 16);
        rs.gen = reinterpret_cast<unsigned *>(words + 17);
        rs.abort = words + 18;
        // a negative wait limit (a test hook) makes every barrier wait give up at once
        rs.timeout = b->wait_limit < 0 ? 0ull : (unsigned long long)(seconds * khz * 1000.0);
        rs.j0 = 0;
        rs.nsteps = nsteps;
        const ShotDesc *desc = g.d_desc;
        BatchItems items = g.items;
        void *args[] = {&desc, &items, &rs};
        if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kVariants[g.variant].run[g.kind]),
                                       dim3(g.run_grid), dim3(g.threads), args, 0, b->stream) != hipSuccess)
            return WAVE_EHIP;
    }
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

// Schedule 1: each shot's steps on one of the K streams with the shot's own
// kernel; the contexts' bookkeeping advances as the launches are enqueued.
// The shots of each stream: largest shots first, each to the stream with
// the least work so far (work = cells per step), so the streams end close
// together.
std::vector<std::vector<size_t>> stream_shots(const wave_batch *b)
{
    const size_t K = b->aux.size();
    std::vector<size_t> order(b->ctx.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = i;
    auto cells = [&](size_t i) {
        const wave_params_t &p = b->ctx[i]->p;
        return (double)p.nx * p.ny * p.nz;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cells(x) > cells(y); });
    std::vector<double> load(K, 0.0);
    std::vector<std::vector<size_t>> out(K);
    for (const size_t i : order) {
        const size_t k = std::min_element(load.begin(), load.end()) - load.begin();
        load[k] += cells(i);
        out[k].push_back(i);
    }
    return out;
}

// Every step of the listed shots on stream k, shot after shot.
int enqueue_stream(wave_batch *b, size_t k, const std::vector<size_t> &shots, int nsteps,
                   const float *const *src_dev)
{
    for (const size_t i : shots) {
        wave_ctx *c = b->ctx[i];
        hipStream_t saved = c->stream;
        c->stream = b->aux[k];
        const float *src = src_dev ? src_dev[i] : nullptr;
        int rc = WAVE_OK;
        for (int j = 0; j < nsteps && rc == WAVE_OK; ++j)
            rc = launch_step(c, src ? src + j : nullptr, 0.f);
        c->stream = saved;
        if (rc != WAVE_OK)
            return rc;
    }
    return WAVE_OK;
}

// Fork the streams that have shots from the batch stream (before their
// work) or join them back into it (after).
int fork_streams(wave_batch *b, const std::vector<std::vector<size_t>> &per)
{
    if (hipEventRecord(b->ev[0], b->stream) != hipSuccess)
        return WAVE_EHIP;
    for (size_t k = 0; k < per.size(); ++k)
        if (!per[k].empty() && hipStreamWaitEvent(b->aux[k], b->ev[0], 0) != hipSuccess)
            return WAVE_EHIP;
    return WAVE_OK;
}

int join_streams(wave_batch *b, const std::vector<std::vector<size_t>> &per)
{
    for (size_t k = 0; k < per.size(); ++k)
        if (!per[k].empty() && (hipEventRecord(b->ev[1 + k], b->aux[k]) != hipSuccess ||
                                hipStreamWaitEvent(b->stream, b->ev[1 + k], 0) != hipSuccess))
            return WAVE_EHIP;
    return WAVE_OK;
}

// Eager launches: one step of each stream's current shot at a time, round
// robin, so that every stream has work queued while the host is still
// launching (a stream's whole share first fills the launch queue and leaves
// the other streams idle).
int batch_enqueue_streams(wave_batch *b, int nsteps, const float *const *src_dev)
{
    const auto per = stream_shots(b);
    if (fork_streams(b, per) != WAVE_OK)
        return WAVE_EHIP;
    const size_t K = per.size();
    std::vector<size_t> pos(K, 0);
    std::vector<int> step(K, 0);
    for (bool more = nsteps > 0; more;) {
        more = false;
        for (size_t k = 0; k < K; ++k) {
            if (pos[k] >= per[k].size())
                continue;
            more = true;
            const size_t i = per[k][pos[k]];
            wave_ctx *c = b->ctx[i];
            hipStream_t saved = c->stream;
            c->stream = b->aux[k];
            const float *src = src_dev ? src_dev[i] : nullptr;
            const int rc = launch_step(c, src ? src + step[k] : nullptr, 0.f);
            c->stream = saved;
            if (rc != WAVE_OK)
                return rc;
            if (++step[k] == nsteps) {
                step[k] = 0;
                ++pos[k];
            }
        }
    }
    return join_streams(b, per);
}

// Schedule 1 under graph replay: capture each stream's launches as a graph
// of its own (the context bookkeeping advances as in an eager run).
int capture_stream_graphs(wave_batch *b, int nsteps, const float *const *src_dev)
{
    const auto per = stream_shots(b);
    b->sgraph.assign(per.size(), nullptr);
    b->sexec.assign(per.size(), nullptr);
    for (size_t k = 0; k < per.size(); ++k) {
        if (per[k].empty())
            continue;
        if (hipStreamBeginCapture(b->aux[k], hipStreamCaptureModeThreadLocal) != hipSuccess)
            return WAVE_EHIP;
        const int rc = enqueue_stream(b, k, per[k], nsteps, src_dev);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->aux[k], &g);
        if (rc != WAVE_OK || e != hipSuccess || !g) {
            if (g)
                (void)hipGraphDestroy(g);
            return WAVE_EHIP;
        }
        b->sgraph[k] = g;
        if (hipGraphInstantiate(&b->sexec[k], g, nullptr, nullptr, 0) != hipSuccess) {
            b->sexec[k] = nullptr;
            return WAVE_EHIP;
        }
    }
    return WAVE_OK;
}

// Replay the per-stream graphs between a fork and a join.
int launch_stream_graphs(wave_batch *b)
{
    const auto per = stream_shots(b);
    if (fork_streams(b, per) != WAVE_OK)
        return WAVE_EHIP;
    for (size_t k = 0; k < per.size(); ++k)
        if (!per[k].empty() && hipGraphLaunch(b->sexec[k], b->aux[k]) != hipSuccess)
            return WAVE_EHIP;
    return join_streams(b, per);
}

int batch_enqueue(wave_batch *b, int nsteps)
{
    for (auto &g : b->groups)
        hipLaunchKernelGGL(clear_counters, dim3(1), dim3(64), 0, b->stream, g.items.counters);
    for (int j = 0; j < nsteps; ++j)
        for (auto &g : b->groups) {
            const BatchKernel k = kVariants[g.variant].batch[g.kind];
            hipLaunchKernelGGL(k, dim3(g.grid), dim3(g.threads), 0, b->stream,
                               (const ShotDesc *)g.d_desc, g.items, j);
        }
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

}  // namespace

extern "C" {

int wave_layout(int32_t nx, int32_t ny, int32_t nz, int32_t dtype, wave_layout_t *out)
{
    if (!out || nx < 1 || ny < 1 || nz < 1)
        return WAVE_EINVAL;
    if (dtype < WAVE_F32 || dtype >= kNumKinds)
        return WAVE_EINVAL;
    const int64_t eb = elem_bytes(dtype);
    const int64_t align = kRowAlignBytes / eb;
    wave_layout_t l;
    const int64_t nxq = (nx + 3) / 4;
    l.x_offset = align;
    l.pitch_x = round_up(align + 4 * nxq + 4, align);
    l.rows = int64_t(ny) + 2 * kGhost;
    l.planes = int64_t(nz) + 2 * kGhost;
    l.plane = l.pitch_x * l.rows;
    // one plane is addressed through one buffer resource (32-bit size)
    if (l.plane * eb >= (int64_t(1) << 31))
        return WAVE_EINVAL;
    l.elems = l.plane * l.planes;
    l.bytes = l.elems * eb;
    *out = l;
    return WAVE_OK;
}

int wave_init(wave_ctx **out, const wave_params_t *p, const void *k, void *u_cur, void *u_prev,
              const int32_t *src_zyx, const int32_t *rec_zyx, int32_t nrec, void *stream)
{
    if (!out)
        return WAVE_EINVAL;
    *out = nullptr;
    if (!p || !k || !u_cur || !u_prev || u_cur == u_prev || nrec < 0 || (nrec > 0 && !rec_zyx))
        return WAVE_EINVAL;
    // 16-byte (FP32) / 8-byte (16-bit) cell groups need aligned fields
    if ((reinterpret_cast<uintptr_t>(k) | reinterpret_cast<uintptr_t>(u_cur) |
         reinterpret_cast<uintptr_t>(u_prev)) & 15u)
        return WAVE_EINVAL;
    wave_layout_t lay, lay32;
    if (wave_layout(p->nx, p->ny, p->nz, p->dtype, &lay) != WAVE_OK ||
        wave_layout(p->nx, p->ny, p->nz, WAVE_F32, &lay32) != WAVE_OK)
        return WAVE_EINVAL;
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz))
        return WAVE_EINVAL;
    if (p->sponge_width < 0 || !std::isfinite(p->sponge_alpha) || p->sponge_alpha < 0.0)
        return WAVE_EINVAL;
    const int dims[3] = {p->nz, p->ny, p->nx};
    if (src_zyx)
        for (int a = 0; a < 3; ++a)
            if (src_zyx[a] < 0 || src_zyx[a] >= dims[a])
                return WAVE_EINVAL;
    for (int32_t r = 0; r < nrec; ++r)
        for (int a = 0; a < 3; ++a)
            if (rec_zyx[3 * r + a] < 0 || rec_zyx[3 * r + a] >= dims[a])
                return WAVE_EINVAL;

    wave_ctx *c = new (std::nothrow) wave_ctx();
    if (!c)
        return WAVE_ENOMEM;
    c->p = *p;
    c->lay = lay;
    c->lay32 = lay32;
    c->cache_resident = p->dtype == WAVE_F32 && fits_in_cache(p->nx, p->ny, p->nz);
    c->stream = static_cast<hipStream_t>(stream);
    c->k = k;
    c->buf0 = c->cur = u_cur;
    c->buf1 = c->prev = u_prev;
    if (src_zyx)
        for (int a = 0; a < 3; ++a)
            c->src[a] = src_zyx[a];
    c->nrec = nrec;
    c->rec.assign(rec_zyx, rec_zyx + 3 * (size_t)nrec);

    const double ih2[3] = {1.0 / (p->dx * p->dx), 1.0 / (p->dy * p->dy), 1.0 / (p->dz * p->dz)};
    c->coefs.ctr = float(kC0 * (ih2[0] + ih2[1] + ih2[2]));
    for (int m = 0; m < 4; ++m) {
        c->coefs.cx[m] = float(kCm[m] * ih2[0]);
        c->coefs.cy[m] = float(kCm[m] * ih2[1]);
        c->coefs.cz[m] = float(kCm[m] * ih2[2]);
    }

    auto bail = [&](int code) {
        free_device(c);
        delete c;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess)
        return bail(WAVE_EHIP);
    // the device address of the fixed scratch array, once per device
    {
        int *sp = nullptr;
        if (scratch_for(c->device, &sp) != WAVE_OK) {
            (void)hipGetLastError();
            return bail(WAVE_EHIP);
        }
    }

    // sponge profiles
    std::vector<float> g;
    float **dst[3] = {&c->gx, &c->gy, &c->gz};
    const int n3[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        sponge_profile(n3[a], p->sponge_width, p->sponge_alpha, g);
        if (hipMalloc(dst[a], sizeof(float) * g.size()) != hipSuccess)
            return bail(WAVE_ENOMEM);
        if (hipMemcpy(*dst[a], g.data(), sizeof(float) * g.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(WAVE_EHIP);
    }
    // receiver offsets in receiver order
    {
        std::vector<long long> off(std::max(nrec, 1));
        for (int r = 0; r < nrec; ++r)
            off[r] = elem_offset(lay, c->rec[3 * r], c->rec[3 * r + 1], c->rec[3 * r + 2]);
        if (hipMalloc(&c->rec_off_all, sizeof(long long) * off.size()) != hipSuccess)
            return bail(WAVE_ENOMEM);
        if (hipMemcpy(c->rec_off_all, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(WAVE_EHIP);
    }
    if (hipMalloc(&c->ring, 8 * sizeof(int)) != hipSuccess)
        return bail(WAVE_ENOMEM);
    if (hipMemsetAsync(c->ring, 0, 8 * sizeof(int), c->stream) != hipSuccess)
        return bail(WAVE_EHIP);
    plan_launch(c);
    if (build_receiver_tables(c) != WAVE_OK)
        return bail(WAVE_EHIP);

    // stability: max(k) * symbol_max * sum 1/h^2 <= 4 (k is FP32 in the FP32 layout)
    unsigned *d = nullptr;
    unsigned init[3] = {0u, 0x7f800000u, 0u}, res[3];
    if (hipMalloc(&d, sizeof(init)) != hipSuccess)
        return bail(WAVE_ENOMEM);
    bool ok = hipMemcpyAsync(d, init, sizeof(init), hipMemcpyHostToDevice, c->stream) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_range, dim3(1024), dim3(256), 0, c->stream, (const float *)k, p->nx,
                           p->ny, p->nz, int(lay32.pitch_x), int(lay32.x_offset),
                           (long long)lay32.plane, d);
        ok = hipGetLastError() == hipSuccess &&
             hipMemcpyAsync(res, d, sizeof(res), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
             hipStreamSynchronize(c->stream) == hipSuccess;
    }
    (void)hipFree(d);
    if (!ok)
        return bail(WAVE_EHIP);
    if (res[2])
        return bail(WAVE_EINVAL);
    float kmax;
    std::memcpy(&kmax, &res[0], sizeof(float));
    if (double(kmax) * kSymbolMax * (ih2[0] + ih2[1] + ih2[2]) > 4.0)
        return bail(WAVE_EUNSTABLE);

    // 16-bit storage: the library keeps its own k, scaled by a power of two
    // so that max(k) lands below 2^14
    if (p->dtype != WAVE_F32) {
        int ex = 0;
        if (kmax > 0.f)
            (void)std::frexp(kmax, &ex);
        const int ek = kmax > 0.f ? ex - kScaledTopExp : 0;
        c->k_scale = std::ldexp(1.f, ek);
        if (hipMalloc(&c->k16, lay.bytes) != hipSuccess)
            return bail(WAVE_ENOMEM);
        if (hipMemsetAsync(c->k16, 0, lay.bytes, c->stream) != hipSuccess)
            return bail(WAVE_EHIP);
        if (launch_convert(c->stream, WAVE_F32, p->dtype, k, c->k16, p->nx, p->ny, p->nz, lay32, lay,
                           std::ldexp(1.f, -ek), nullptr, 0) != WAVE_OK)
            return bail(WAVE_EHIP);
        if (hipStreamSynchronize(c->stream) != hipSuccess)
            return bail(WAVE_EHIP);
        c->k = c->k16;
    }
    // u-and-change storage: d^0 = u^0 - u^{-1} = 0 (both start at zero)
    if (is_uv(p->dtype)) {
        if (hipMalloc(&c->dbuf, lay.bytes) != hipSuccess)
            return bail(WAVE_ENOMEM);
        if (hipMemsetAsync(c->dbuf, 0, lay.bytes, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return bail(WAVE_EHIP);
    }

    *out = c;
    return WAVE_OK;
}

int wave_record(wave_ctx *ctx, float *traces_dev, int32_t nt_capacity)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (traces_dev && nt_capacity < 0)
        return fail(ctx, WAVE_EINVAL, "negative trace capacity");
    ctx->traces = traces_dev;
    ctx->trace_cap = traces_dev ? nt_capacity : 0;
    return WAVE_OK;
}

int wave_step(wave_ctx *ctx, float src_value)
{
    if (!ctx)
        return WAVE_EINVAL;
    int rc = check_trace_room(ctx, 1);
    if (rc != WAVE_OK)
        return rc;
    return launch_step(ctx, nullptr, src_value);
}

int wave_run(wave_ctx *ctx, int32_t nsteps, const float *src_dev)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (nsteps < 0)
        return fail(ctx, WAVE_EINVAL, "nsteps < 0");
    int rc = check_trace_room(ctx, nsteps);
    if (rc != WAVE_OK)
        return rc;
    if (ctx->use_graph && nsteps > 0) {
        wave_ctx::RunGraph &g = ctx->rg;
        const bool same = g.exec && g.step0 == ctx->step && g.nsteps == nsteps && g.src == src_dev &&
                          g.traces == ctx->traces && g.cur == ctx->cur && g.prev == ctx->prev;
        if (!same) {
            // capture this run's launches (the host bookkeeping advances as
            // in an eager run), then replay them
            drop_run_graph(ctx);
            const int64_t step0 = ctx->step;
            void *cur0 = ctx->cur, *prev0 = ctx->prev;
            HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            int lrc = WAVE_OK;
            for (int32_t j = 0; j < nsteps && lrc == WAVE_OK; ++j)
                lrc = launch_step(ctx, src_dev ? src_dev + j : nullptr, 0.0f);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
            if (lrc != WAVE_OK || ec != hipSuccess) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                ctx->step = step0;
                ctx->cur = cur0;
                ctx->prev = prev0;
                return lrc != WAVE_OK ? lrc : fail(ctx, WAVE_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
            }
            hipGraphExec_t exec = nullptr;
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                ctx->step = step0;
                ctx->cur = cur0;
                ctx->prev = prev0;
                return fail(ctx, WAVE_EHIP, "graph instantiation failed");
            }
            g.graph = graph;
            g.exec = exec;
            g.step0 = step0;
            g.nsteps = nsteps;
            g.src = src_dev;
            g.traces = ctx->traces;
            g.cur = cur0;
            g.prev = prev0;
            HIP_TRY(ctx, hipGraphLaunch(exec, ctx->stream));
            return WAVE_OK;
        }
        HIP_TRY(ctx, hipGraphLaunch(g.exec, ctx->stream));
        // the same bookkeeping as the captured launches
        if (nsteps & 1)
            std::swap(ctx->cur, ctx->prev);
        ctx->step += nsteps;
        return WAVE_OK;
    }
    for (int32_t j = 0; j < nsteps; ++j) {
        rc = launch_step(ctx, src_dev ? src_dev + j : nullptr, 0.0f);
        if (rc != WAVE_OK)
            return rc;
    }
    return WAVE_OK;
}

int wave_set_graph(wave_ctx *ctx, int32_t on)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (on && !ctx->stream)
        return fail(ctx, WAVE_EINVAL, "graph replay needs a stream other than the legacy default stream");
    ctx->use_graph = on != 0;
    if (!ctx->use_graph)
        drop_run_graph(ctx);
    return WAVE_OK;
}

int wave_fields(const wave_ctx *ctx, void **cur, void **prev, int64_t *step)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (cur)
        *cur = ctx->cur;
    if (prev)
        *prev = ctx->prev;
    if (step)
        *step = ctx->step;
    return WAVE_OK;
}

int wave_export(wave_ctx *ctx, int32_t which, float *dst)
{
    if (!ctx)
        return WAVE_EINVAL;
    if ((which != 0 && which != 1) || !dst || (reinterpret_cast<uintptr_t>(dst) & 15u))
        return fail(ctx, WAVE_EINVAL, "wave_export: which must be 0 or 1 and dst a 16-byte aligned field");
    const void *src = which == 0 ? ctx->cur : ctx->prev;
    const int slot = int((ctx->step + (which == 0 ? 0 : 3)) & 3);
    const int kind = ctx->p.dtype;
    const int rc = launch_convert(ctx->stream, kind, WAVE_F32, src, dst, ctx->p.nx, ctx->p.ny,
                                  ctx->p.nz, ctx->lay, ctx->lay32, 1.f,
                                  kind == WAVE_F32 ? nullptr : ctx->ring, slot);
    return rc == WAVE_OK ? WAVE_OK : fail(ctx, rc, "export launch failed");
}

int wave_reset(wave_ctx *ctx)
{
    if (!ctx)
        return WAVE_EINVAL;
    ctx->cur = ctx->buf0;
    ctx->prev = ctx->buf1;
    ctx->step = 0;
    HIP_TRY(ctx, hipMemsetAsync(ctx->ring, 0, 8 * sizeof(int), ctx->stream));
    if (ctx->dbuf)
        HIP_TRY(ctx, hipMemsetAsync(ctx->dbuf, 0, ctx->lay.bytes, ctx->stream));
    return WAVE_OK;
}

int wave_set_stream(wave_ctx *ctx, void *stream)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (!stream && ctx->use_graph)
        return fail(ctx, WAVE_EINVAL, "graph replay is on: the stream cannot be the legacy default stream");
    ctx->stream = static_cast<hipStream_t>(stream);
    return WAVE_OK;
}

int wave_configure(wave_ctx *ctx, int32_t variant, int32_t zchunk)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (variant < 0 || variant >= kNumVariants || zchunk < 0)
        return fail(ctx, WAVE_EINVAL, "unknown variant %d or negative z-chunk %d", variant, zchunk);
    ctx->variant = variant;
    ctx->zchunk = zchunk;
    drop_run_graph(ctx);  // its launches name the old tables
    plan_launch(ctx);
    return build_receiver_tables(ctx);
}

int32_t wave_variant_count(void) { return kNumVariants; }

const char *wave_variant_name(int32_t variant)
{
    if (variant < 0 || variant >= kNumVariants)
        return nullptr;
    return kVariants[variant].name;
}

int wave_config(const wave_ctx *ctx, int32_t *variant, int32_t *zchunk, int32_t *workgroups)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (variant)
        *variant = ctx->v_used;
    if (zchunk)
        *zchunk = ctx->zc_used;
    if (workgroups)
        *workgroups = ctx->nwg;
    return WAVE_OK;
}

int wave_sync(wave_ctx *ctx)
{
    if (!ctx)
        return WAVE_EINVAL;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipGetLastError());
    return WAVE_OK;
}

int wave_destroy(wave_ctx *ctx)
{
    if (!ctx)
        return WAVE_OK;
    free_device(ctx);
    delete ctx;
    return WAVE_OK;
}

int wave_forward_checkpointed(wave_ctx *ctx, int32_t nt, const float *src_dev, int32_t every)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (ctx->p.dtype != WAVE_F32)
        return fail(ctx, WAVE_EINVAL, "the gradient is available for FP32 storage only");
    if (nt < 1 || every < 0)
        return fail(ctx, WAVE_EINVAL, "nt must be >= 1 and every >= 0");
    int rc = check_trace_room(ctx, nt);
    if (rc != WAVE_OK)
        return rc;
    int C = every > 0 ? std::min(every, nt) : auto_segment(ctx, nt);
    if (C < 1)
        return fail(ctx, WAVE_ENOMEM, "not enough device memory for the checkpoints of %d steps", nt);
    wave_grad_state &g = ctx->g;
    const int nseg = (nt + C - 1) / C;
    const size_t levels = 2 * (size_t)nseg + (size_t)C;
    g.nt = 0;  // invalid until the run is enqueued
    if (levels > g.slab_levels) {
        free_dev(g.slab);
        g.slab_levels = 0;
        if (hipMalloc(&g.slab, levels * level_bytes(ctx)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, WAVE_ENOMEM, "cannot allocate %zu field levels (%.2f GB)", levels,
                        levels * double(level_bytes(ctx)) / 1e9);
        }
        g.slab_levels = levels;
        // ghost cells stay zero: steps write interior cells only
        HIP_TRY(ctx, hipMemsetAsync(g.slab, 0, levels * level_bytes(ctx), ctx->stream));
    }
    if (src_dev) {
        if (nt > g.src_cap) {
            free_dev(g.src);
            g.src_cap = 0;
            HIP_TRY(ctx, hipMalloc(&g.src, sizeof(float) * (size_t)nt));
            g.src_cap = nt;
        }
        HIP_TRY(ctx, hipMemcpyAsync(g.src, src_dev, sizeof(float) * (size_t)nt,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    }
    g.has_src = src_dev != nullptr;
    g.step0 = ctx->step;
    g.every = C;
    g.nseg = nseg;
    g.held = -1;

    const size_t lb = level_bytes(ctx);
    for (int seg = 0; seg < nseg; ++seg) {
        const int64_t c0 = (int64_t)seg * C;
        const int len = int(std::min<int64_t>(C, nt - c0));
        HIP_TRY(ctx, hipMemcpyAsync(level_ptr(ctx, seg, c0 - 1), ctx->prev, lb, hipMemcpyDeviceToDevice,
                                    ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(level_ptr(ctx, seg, c0), ctx->cur, lb, hipMemcpyDeviceToDevice,
                                    ctx->stream));
        if (seg + 1 < nseg) {
            for (int j = 0; j < len; ++j) {
                rc = launch_step(ctx, g.has_src ? g.src + c0 + j : nullptr, 0.f);
                if (rc != WAVE_OK)
                    return rc;
            }
        } else {
            // the last segment keeps its levels for the adjoint run
            rc = forward_segment(ctx, seg, len, true);
            if (rc != WAVE_OK)
                return rc;
            HIP_TRY(ctx, hipMemcpyAsync(ctx->prev, level_ptr(ctx, seg, c0 + len - 1), lb,
                                        hipMemcpyDeviceToDevice, ctx->stream));
            HIP_TRY(ctx, hipMemcpyAsync(ctx->cur, level_ptr(ctx, seg, c0 + len), lb,
                                        hipMemcpyDeviceToDevice, ctx->stream));
            ctx->step += len;
        }
    }
    g.nt = nt;
    return WAVE_OK;
}

namespace {

// The adjoint run of the last checkpointed forward run, leaving dJ/dk in the
// FP64 accumulator g.acc (field layout).  With src_term, the source values
// are taken to scale with k at the source cell, and their derivative is
// added there.
int adjoint_run(wave_ctx *ctx, const float *trace_grad_dev, bool src_term)
{
    wave_grad_state &g = ctx->g;
    int rc = build_receiver_cells(ctx);
    if (rc != WAVE_OK)
        return rc;
    const size_t lb = level_bytes(ctx);
    const size_t ab = (size_t)ctx->lay.elems * sizeof(double);
    for (int i = 0; i < 2; ++i)
        if (!g.phi[i]) {
            HIP_TRY(ctx, hipMalloc(&g.phi[i], lb));
        }
    if (!g.acc) {
        HIP_TRY(ctx, hipMalloc(&g.acc, ab));
    }
    HIP_TRY(ctx, hipMemsetAsync(g.phi[0], 0, lb, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(g.phi[1], 0, lb, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(g.acc, 0, ab, ctx->stream));

    // the source cell's thread in inject_receivers: the receiver cell that is
    // also the source cell, else one past the receiver cells
    src_term = src_term && g.has_src && ctx->src[0] >= 0;
    long long src_off = 0;
    int src_thread = g.ncells;
    if (src_term) {
        src_off = elem_offset(ctx->lay, ctx->src[0], ctx->src[1], ctx->src[2]);
        for (int i = 0; i < g.ncells; ++i)
            if (g.cell_off_host[i] == src_off)
                src_thread = i;
    }

    const Geo geo = adjoint_geo(ctx);
    // + K R^T (dJ/d traces, row m-1) into phi^m (and the source-cell term)
    auto inject = [&](void *phi, int m) -> int {
        const int threads = g.ncells + (src_term ? 1 : 0);
        if (threads > 0) {
            hipLaunchKernelGGL(inject_receivers, dim3((threads + 255) / 256), dim3(256), 0, ctx->stream,
                               static_cast<float *>(phi), static_cast<const float *>(ctx->k), g.cell_off,
                               g.cell_start, g.cell_rec, g.ncells,
                               g.ncells > 0 ? trace_grad_dev + (size_t)(m - 1) * ctx->nrec : nullptr,
                               src_term ? g.src + (m - 1) : nullptr, src_off, src_thread, g.acc);
            HIP_TRY(ctx, hipGetLastError());
        }
        return WAVE_OK;
    };
    // the level a^l, recomputing its segment from the checkpoint if needed
    auto level = [&](int64_t l, const void **out) -> int {
        const int seg = int(l / g.every);
        if (g.held != seg) {
            const int64_t c0 = (int64_t)seg * g.every;
            const int r = forward_segment(ctx, seg, int(std::min<int64_t>(g.every, g.nt - c0)) - 1, false);
            if (r != WAVE_OK)
                return r;
        }
        *out = level_ptr(ctx, seg, l);
        return WAVE_OK;
    };
    const void *lev = nullptr;
    void *A = g.phi[0], *B = g.phi[1];  // phi^{m+1}, phi^{m+2}
    if (ctx->fuse_adjoint) {
        // phi^nt, then for m = nt .. 2 one pass makes phi^{m-1} and adds the
        // imaging term of phi^m; the term of phi^1 closes the sum
        rc = enqueue_adjoint(ctx, geo, kAdj, A, B, B, nullptr);
        if (rc == WAVE_OK)
            rc = inject(B, g.nt);
        if (rc != WAVE_OK)
            return rc;
        std::swap(A, B);  // A = phi^m, B = phi^{m+1}
        for (int m = g.nt; m >= 2; --m) {
            if ((rc = level(m - 1, &lev)) != WAVE_OK)
                return rc;
            rc = enqueue_adjoint(ctx, geo, kFus, A, B, B, g.acc, lev);
            if (rc == WAVE_OK)
                rc = inject(B, m - 1);
            if (rc != WAVE_OK)
                return rc;
            std::swap(A, B);
        }
        if ((rc = level(0, &lev)) != WAVE_OK)
            return rc;
        if ((rc = enqueue_adjoint(ctx, geo, kImg, lev, A, nullptr, g.acc)) != WAVE_OK)
            return rc;
    } else {
        for (int m = g.nt; m >= 1; --m) {
            // phi^m = 2 G phi^{m+1} + K L G phi^{m+1} - G^2 phi^{m+2}, over phi^{m+2}
            rc = enqueue_adjoint(ctx, geo, kAdj, A, B, B, nullptr);
            if (rc != WAVE_OK)
                return rc;
            std::swap(A, B);
            if ((rc = inject(A, m)) != WAVE_OK)
                return rc;
            // grad += (G phi^m / k) L a^{m-1}
            if ((rc = level(m - 1, &lev)) != WAVE_OK)
                return rc;
            if ((rc = enqueue_adjoint(ctx, geo, kImg, lev, A, nullptr, g.acc)) != WAVE_OK)
                return rc;
        }
    }
    return WAVE_OK;
}

// dJ/dk (v == nullptr) or dJ/dv (k = (v dt)^2) from the accumulator into a
// dense FP64 array.
int adjoint_output(wave_ctx *ctx, double *grad_dev, int32_t accumulate, const float *v_dev, double dt)
{
    const long long n = (long long)ctx->p.nx * ctx->p.ny * ctx->p.nz;
    hipLaunchKernelGGL(grad_to_dense, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256),
                       0, ctx->stream, ctx->g.acc, grad_dev, ctx->p.nx, ctx->p.ny, ctx->p.nz,
                       int(ctx->lay.pitch_x), int(ctx->lay.x_offset), (long long)ctx->lay.plane,
                       accumulate ? 1 : 0, v_dev, 2.0 * dt * dt);
    HIP_TRY(ctx, hipGetLastError());
    return WAVE_OK;
}

int adjoint_checks(wave_ctx *ctx, const float *trace_grad_dev, const double *grad_dev)
{
    if (ctx->g.nt < 1)
        return fail(ctx, WAVE_ESTATE, "the adjoint run needs a preceding wave_forward_checkpointed");
    if (!grad_dev || (ctx->nrec > 0 && !trace_grad_dev))
        return fail(ctx, WAVE_EINVAL, "adjoint run: grad and (with receivers) trace_grad are required");
    return WAVE_OK;
}

}  // namespace

int wave_adjoint(wave_ctx *ctx, const float *trace_grad_dev, double *grad_dev, int32_t accumulate)
{
    if (!ctx)
        return WAVE_EINVAL;
    int rc = adjoint_checks(ctx, trace_grad_dev, grad_dev);
    if (rc == WAVE_OK)
        rc = adjoint_run(ctx, trace_grad_dev, false);
    if (rc == WAVE_OK)
        rc = adjoint_output(ctx, grad_dev, accumulate, nullptr, 0.0);
    return rc;
}

int wave_adjoint_velocity(wave_ctx *ctx, const float *trace_grad_dev, const float *v_dev, double dt,
                          int32_t source_scales_with_k, double *grad_v_dev, int32_t accumulate)
{
    if (!ctx)
        return WAVE_EINVAL;
    if (!v_dev || !(std::isfinite(dt) && dt > 0.0))
        return fail(ctx, WAVE_EINVAL, "wave_adjoint_velocity: v is required and dt must be > 0");
    int rc = adjoint_checks(ctx, trace_grad_dev, grad_v_dev);
    if (rc == WAVE_OK)
        rc = adjoint_run(ctx, trace_grad_dev, source_scales_with_k != 0);
    if (rc == WAVE_OK)
        rc = adjoint_output(ctx, grad_v_dev, accumulate, v_dev, dt);
    return rc;
}

int wave_velocity_to_k(const float *v_dev, int64_t n, double dt, float *k_dev, void *stream)
{
    if (!v_dev || !k_dev || n < 0 || !(std::isfinite(dt) && dt > 0.0))
        return WAVE_EINVAL;
    if (n == 0)
        return WAVE_OK;
    hipLaunchKernelGGL(velocity_to_k, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), v_dev, (long long)n, dt, k_dev);
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

int wave_check(wave_ctx *ctx, int64_t *field_nonfinite, int64_t *trace_nonfinite)
{
    if (!ctx)
        return WAVE_EINVAL;
    int *d = nullptr;
    int h[2] = {0, 0};
    HIP_TRY(ctx, hipMalloc(&d, 2 * sizeof(int)));
    const long long cells = (long long)ctx->p.nx * ctx->p.ny * ctx->p.nz;
    const long long nt = (ctx->traces && ctx->nrec > 0) ? std::min<long long>(ctx->step, ctx->trace_cap) : 0;
    bool ok = hipMemsetAsync(d, 0, 2 * sizeof(int), ctx->stream) == hipSuccess;
    if (ok) {
        const dim3 g((unsigned)std::min<long long>((std::max(cells, nt * ctx->nrec) + 255) / 256, 4096));
        hipLaunchKernelGGL(count_nonfinite, g, dim3(256), 0, ctx->stream, (const void *)ctx->cur,
                           ctx->p.dtype, ctx->p.nx, ctx->p.ny, ctx->p.nz, int(ctx->lay.pitch_x),
                           int(ctx->lay.x_offset), (long long)ctx->lay.plane, (const float *)ctx->traces,
                           nt * ctx->nrec, d);
        ok = hipGetLastError() == hipSuccess &&
             hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
             hipStreamSynchronize(ctx->stream) == hipSuccess;
    }
    (void)hipFree(d);
    if (!ok)
        return fail(ctx, WAVE_EHIP, "wave_check failed");
    if (field_nonfinite)
        *field_nonfinite = h[0];
    if (trace_nonfinite)
        *trace_nonfinite = h[1];
    return WAVE_OK;
}

int wave_set_adjoint_fusion(wave_ctx *ctx, int32_t on)
{
    if (!ctx)
        return WAVE_EINVAL;
    ctx->fuse_adjoint = on != 0;
    return WAVE_OK;
}

int wave_grad_info(const wave_ctx *ctx, int32_t *nt, int32_t *every, int32_t *segments, int64_t *bytes)
{
    if (!ctx)
        return WAVE_EINVAL;
    const wave_grad_state &g = ctx->g;
    if (nt)
        *nt = g.nt;
    if (every)
        *every = g.every;
    if (segments)
        *segments = g.nseg;
    if (bytes)
        *bytes = int64_t(g.slab_levels * level_bytes(ctx));
    return WAVE_OK;
}

int wave_check_noalloc(wave_ctx *ctx, int64_t *field_nonfinite, int64_t *trace_nonfinite)
{
    if (!ctx)
        return WAVE_EINVAL;
    constexpr int kCounters = 2;
    static_assert(kCounters <= kScratchInts, "the counters must fit in the scratch array");
    int *d = nullptr;
    if (scratch_for(ctx->device, &d) != WAVE_OK)
        return fail(ctx, WAVE_EHIP, "wave_check_noalloc: the scratch array's address is not available");
    int h[kCounters] = {0, 0};
    const long long cells = (long long)ctx->p.nx * ctx->p.ny * ctx->p.nz;
    const long long nt = (ctx->traces && ctx->nrec > 0) ? std::min<long long>(ctx->step, ctx->trace_cap) : 0;
    // the array keeps the last call's counts: clear them with a kernel first
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(256), 0, ctx->stream, d, (long long)kCounters);
    const dim3 g((unsigned)std::min<long long>((std::max(cells, nt * ctx->nrec) + 255) / 256, 4096));
    hipLaunchKernelGGL(count_nonfinite, g, dim3(256), 0, ctx->stream, (const void *)ctx->cur, ctx->p.dtype,
                       ctx->p.nx, ctx->p.ny, ctx->p.nz, int(ctx->lay.pitch_x), int(ctx->lay.x_offset),
                       (long long)ctx->lay.plane, (const float *)ctx->traces, nt * ctx->nrec, d);
    const bool ok = hipGetLastError() == hipSuccess &&
                    hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
                    hipStreamSynchronize(ctx->stream) == hipSuccess;
    if (!ok)
        return fail(ctx, WAVE_EHIP, "wave_check_noalloc failed");
    if (field_nonfinite)
        *field_nonfinite = h[0];
    if (trace_nonfinite)
        *trace_nonfinite = h[1];
    return WAVE_OK;
}

int wave_misfit(const float *traces_dev, const float *observed_dev, int64_t n, float *residual_dev,
                double *misfit_dev, void *stream)
{
    if (n < 0 || !misfit_dev || (n > 0 && (!traces_dev || !observed_dev)))
        return WAVE_EINVAL;
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), traces_dev,
                       observed_dev, (long long)n, residual_dev, misfit_dev);
    return hipGetLastError() == hipSuccess ? WAVE_OK : WAVE_EHIP;
}

int wave_batch_create(wave_batch **out, wave_ctx *const *ctxs, int32_t nshots, void *stream,
                      int32_t use_graph)
{
    if (!out)
        return WAVE_EINVAL;
    *out = nullptr;
    if (!ctxs || nshots < 1 || (use_graph && !stream))
        return WAVE_EINVAL;
    for (int i = 0; i < nshots; ++i) {
        if (!ctxs[i] || ctxs[i]->v_used == kNaive || is_uv(ctxs[i]->p.dtype))
            return WAVE_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i])
                return WAVE_EINVAL;
    }
    wave_batch *b = new (std::nothrow) wave_batch();
    if (!b)
        return WAVE_ENOMEM;
    b->stream = static_cast<hipStream_t>(stream);
    b->use_graph = use_graph != 0;
    b->ctx.assign(ctxs, ctxs + nshots);
    for (int i = 0; i < nshots; ++i) {
        const wave_ctx *c = ctxs[i];
        b->cfg.insert(b->cfg.end(), {c->v_used, c->zc_used, c->nwg});
        b->points += (long long)c->p.nx * c->p.ny * c->p.nz;
        b->workgroups += c->nwg;
        int gi = -1;
        for (size_t g = 0; g < b->groups.size(); ++g)
            if (b->groups[g].kind == c->p.dtype && b->groups[g].variant == c->v_used)
                gi = int(g);
        if (gi < 0) {
            b->groups.emplace_back();
            gi = int(b->groups.size()) - 1;
            b->groups[gi].kind = c->p.dtype;
            b->groups[gi].variant = c->v_used;
        }
        b->groups[gi].shots.push_back(i);
    }
    int device = 0, cus = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        delete b;
        return WAVE_EHIP;
    }
    for (auto &g : b->groups) {
        const Variant &V = kVariants[g.variant];
        g.threads = V.txv * V.ty;
        // items: every tile/chunk of every shot, shot by shot in spatial
        // order; work = cells the item updates (planes x tile cells within
        // the grid) plus the 8 planes it re-reads
        std::vector<int> ishot, ilid;
        std::vector<double> work;
        for (size_t t = 0; t < g.shots.size(); ++t) {
            const wave_ctx *c = b->ctx[g.shots[t]];
            const int tx = 4 * V.txv, tyr = V.ty * V.ry;
            for (int lid = 0; lid < c->nwg; ++lid) {
                const int ix = lid % c->ntx, rest = lid / c->ntx, iy = rest % c->nty, ch = rest / c->nty;
                const int wx = std::min(tx, c->p.nx - ix * tx), wy = std::min(tyr, c->p.ny - iy * tyr);
                const int wz = std::min(c->zc_used, c->p.nz - ch * c->zc_used);
                ishot.push_back(int(t));
                ilid.push_back(lid);
                work.push_back(double(wx) * wy * (wz + 8));
            }
        }
        g.total = int(ishot.size());
        double wsum = 0.0;
        for (double w : work)
            wsum += w;
        // 8 contiguous ranges of about equal work
        std::vector<int> xs(9, g.total);
        xs[0] = 0;
        double acc = 0.0;
        int part = 1;
        for (int i = 0; i < g.total && part < 8; ++i) {
            acc += work[i];
            while (part < 8 && acc >= wsum * part / 8.0)
                xs[part++] = i + 1;
        }
        // within each range, longest items first (stable: the items of one
        // shot keep their spatial order), so that the end of a step is
        // made of short items
        {
            std::vector<int> order(g.total);
            for (int i = 0; i < g.total; ++i)
                order[i] = i;
            for (int r = 0; r < 8; ++r)
                std::stable_sort(order.begin() + xs[r], order.begin() + xs[r + 1],
                                 [&](int a, int b) { return work[a] > work[b]; });
            std::vector<int> s2(g.total), l2(g.total);
            for (int i = 0; i < g.total; ++i) {
                s2[i] = ishot[order[i]];
                l2[i] = ilid[order[i]];
            }
            ishot.swap(s2);
            ilid.swap(l2);
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V.batch[g.kind], g.threads, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        g.grid = int(round_up(std::min<long long>((long long)per_cu * cus, g.total), 8));
        std::vector<int> blob;
        blob.insert(blob.end(), ishot.begin(), ishot.end());
        blob.insert(blob.end(), ilid.begin(), ilid.end());
        blob.insert(blob.end(), xs.begin(), xs.end());
        blob.insert(blob.end(), 16 + kRunSyncInts, 0);  // tickets [2][8], then the run's barrier words
        g.h_desc.assign(g.shots.size(), ShotDesc{});
        std::memset(g.h_desc.data(), 0, sizeof(ShotDesc) * g.h_desc.size());
        if (hipMalloc(&g.d_desc, sizeof(ShotDesc) * g.shots.size()) != hipSuccess ||
            hipMalloc(&g.d_items, sizeof(int) * blob.size()) != hipSuccess) {
            batch_free(b);
            delete b;
            return WAVE_ENOMEM;
        }
        g.items.shot = g.d_items;
        g.items.lid = g.d_items + g.total;
        g.items.xcd_start = g.d_items + 2 * g.total;
        g.items.counters = g.d_items + 2 * g.total + 9;
        if (hipMemcpy(g.d_items, blob.data(), sizeof(int) * blob.size(), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(g.d_desc, g.h_desc.data(), sizeof(ShotDesc) * g.h_desc.size(),
                      hipMemcpyHostToDevice) != hipSuccess) {
            batch_free(b);
            delete b;
            return WAVE_EHIP;
        }
    }
    *out = b;
    return WAVE_OK;
}

int wave_batch_run(wave_batch *b, int32_t nsteps, const float *const *src_dev)
{
    if (!b)
        return WAVE_EINVAL;
    if (nsteps < 0)
        return bfail(b, WAVE_EINVAL, "nsteps < 0");
    const int64_t n0 = b->ctx[0]->step;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        wave_ctx *c = b->ctx[i];
        if (c->step != n0)
            return bfail(b, WAVE_ESTATE, "shot %zu is at step %lld, shot 0 at %lld", i,
                         (long long)c->step, (long long)n0);
        if (c->v_used != b->cfg[3 * i] || c->zc_used != b->cfg[3 * i + 1] || c->nwg != b->cfg[3 * i + 2])
            return bfail(b, WAVE_ESTATE, "shot %zu was reconfigured after the batch was created", i);
        if (check_trace_room(c, nsteps) != WAVE_OK)
            return bfail(b, WAVE_EINVAL, "shot %zu: %s", i, c->err.c_str());
    }
    if (n0 + nsteps > 0x3fffffff)
        return bfail(b, WAVE_EINVAL, "step counter out of range");
    if (b->schedule == 1) {
        if (nsteps == 0)
            return WAVE_OK;
        std::vector<int64_t> key = {nsteps};
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            const wave_ctx *c = b->ctx[i];
            key.insert(key.end(), {c->step, (int64_t)(uintptr_t)c->cur, (int64_t)(uintptr_t)c->prev,
                                   (int64_t)(uintptr_t)c->traces,
                                   (int64_t)(uintptr_t)(src_dev ? src_dev[i] : nullptr)});
        }
        if (b->use_graph && !b->sexec.empty() && key == b->key) {
            if (launch_stream_graphs(b) != WAVE_OK)
                return bfail(b, WAVE_EHIP, "graph launch failed");
            for (wave_ctx *c : b->ctx) {  // the captured launches' bookkeeping
                c->step += nsteps;
                if (nsteps & 1)
                    std::swap(c->cur, c->prev);
            }
            return WAVE_OK;
        }
        std::vector<std::pair<void *, void *>> roles;
        for (wave_ctx *c : b->ctx)
            roles.push_back({c->cur, c->prev});
        auto restore = [&]() {
            for (size_t i = 0; i < b->ctx.size(); ++i) {
                b->ctx[i]->step = n0;
                b->ctx[i]->cur = roles[i].first;
                b->ctx[i]->prev = roles[i].second;
            }
        };
        if (!b->use_graph) {
            if (batch_enqueue_streams(b, nsteps, src_dev) != WAVE_OK)
                return bfail(b, WAVE_EHIP, "batched launch failed");
            return WAVE_OK;
        }
        // a replaced graph may still be running: wait before destroying it
        if (!b->sexec.empty() && hipStreamSynchronize(b->stream) != hipSuccess)
            return bfail(b, WAVE_EHIP, "stream synchronisation failed");
        drop_batch_graph(b);
        if (capture_stream_graphs(b, nsteps, src_dev) != WAVE_OK) {
            drop_batch_graph(b);
            restore();
            return bfail(b, WAVE_EHIP, "graph capture failed");
        }
        b->key = key;
        if (launch_stream_graphs(b) != WAVE_OK)
            return bfail(b, WAVE_EHIP, "graph launch failed");
        return WAVE_OK;
    }
    // descriptors of this run; upload only what changed (after the work
    // that may still read the old ones)
    bool synced = false;
    for (auto &g : b->groups) {
        std::vector<ShotDesc> d(g.shots.size());
        std::memset(d.data(), 0, sizeof(ShotDesc) * d.size());
        for (size_t t = 0; t < g.shots.size(); ++t) {
            const wave_ctx *c = b->ctx[g.shots[t]];
            d[t].a = make_args(c);
            d[t].traces = (c->traces && c->nrec > 0) ? c->traces : nullptr;
            d[t].nrec = c->nrec;
            d[t].n0 = int(n0);
            d[t].src = src_dev ? src_dev[g.shots[t]] : nullptr;
        }
        if (std::memcmp(d.data(), g.h_desc.data(), sizeof(ShotDesc) * d.size()) != 0) {
            if (!synced) {
                if (hipStreamSynchronize(b->stream) != hipSuccess)
                    return bfail(b, WAVE_EHIP, "stream synchronisation failed");
                synced = true;
            }
            if (hipMemcpy(g.d_desc, d.data(), sizeof(ShotDesc) * d.size(), hipMemcpyHostToDevice) !=
                hipSuccess)
                return bfail(b, WAVE_EHIP, "descriptor upload failed");
            g.h_desc = d;
        }
    }
    if (nsteps > 0 && b->schedule == 3) {
        // one launch per group for the whole run: nothing to capture
        if (run_enqueue(b, nsteps) != WAVE_OK)
            return bfail(b, WAVE_EHIP, "single-launch run failed to start");
    } else if (nsteps > 0) {
        if (b->use_graph) {
            if (b->graph_steps != nsteps) {
                // a replaced graph may still be running: wait before destroying it
                if (b->exec && !synced && hipStreamSynchronize(b->stream) != hipSuccess)
                    return bfail(b, WAVE_EHIP, "stream synchronisation failed");
                if (b->exec)
                    (void)hipGraphExecDestroy(b->exec);
                if (b->graph)
                    (void)hipGraphDestroy(b->graph);
                b->exec = nullptr;
                b->graph = nullptr;
                b->graph_steps = -1;
                if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return bfail(b, WAVE_EHIP, "graph capture could not start");
                const int rc = b->schedule == 2 ? flow_enqueue(b, nsteps) : batch_enqueue(b, nsteps);
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (rc != WAVE_OK || e != hipSuccess || !g) {
                    if (g)
                        (void)hipGraphDestroy(g);
                    return bfail(b, WAVE_EHIP, "graph capture failed");
                }
                if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    b->exec = nullptr;
                    return bfail(b, WAVE_EHIP, "graph instantiation failed");
                }
                b->graph = g;
                b->graph_steps = nsteps;
            }
            if (hipGraphLaunch(b->exec, b->stream) != hipSuccess)
                return bfail(b, WAVE_EHIP, "graph launch failed");
        } else if ((b->schedule == 2 ? flow_enqueue(b, nsteps) : batch_enqueue(b, nsteps)) != WAVE_OK) {
            return bfail(b, WAVE_EHIP, "batched launch failed");
        }
    }
    for (wave_ctx *c : b->ctx) {
        c->step += nsteps;
        if (nsteps & 1) {
            void *t = c->prev;
            c->prev = c->cur;
            c->cur = t;
        }
    }
    return WAVE_OK;
}

int wave_batch_set_schedule(wave_batch *b, int32_t schedule, int32_t nstreams)
{
    if (!b)
        return WAVE_EINVAL;
    if (schedule < 0 || schedule > 3 || (schedule == 1 && (nstreams < 1 || nstreams > 16)))
        return bfail(b, WAVE_EINVAL, "schedule must be 0, 1 with 1..16 streams, 2 or 3");
    if (schedule == 2 && !kFlowScheduleEnabled)
        return bfail(b, WAVE_EINVAL,
                     "schedule 2 is switched off: its first GPU run did not complete and the cause is not known");
    if (schedule == 2)
        for (const auto &g : b->groups)
            if (g.kind != WAVE_F32)
                return bfail(b, WAVE_EINVAL, "schedule 2 runs FP32 shots only");
    if (schedule == 1 && b->use_graph && !b->stream)
        return bfail(b, WAVE_EINVAL, "graph replay needs a stream other than the legacy default stream");
    if (hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, WAVE_EHIP, "stream synchronisation failed");
    drop_batch_graph(b);
    drop_streams(b);
    drop_flow(b);
    b->schedule = 0;
    if (schedule == 2) {
        const int rc = build_flow(b);
        if (rc != WAVE_OK) {
            drop_flow(b);
            return bfail(b, rc, "schedule 2 plan could not be built");
        }
        b->schedule = 2;
    }
    if (schedule == 3) {
        const int rc = build_run(b);
        if (rc != WAVE_OK)
            return bfail(b, rc, rc == WAVE_EINVAL ? "schedule 3 needs cooperative launches, which the device lacks"
                                                  : "schedule 3 plan could not be built");
        b->schedule = 3;
    }
    if (schedule == 1) {
        // on any failure the batch stays on schedule 0 with no streams
        for (int k = 0; k < nstreams; ++k) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                drop_streams(b);
                return bfail(b, WAVE_EHIP, "stream creation failed");
            }
            b->aux.push_back(st);
        }
        for (int k = 0; k <= nstreams; ++k) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                drop_streams(b);
                return bfail(b, WAVE_EHIP, "event creation failed");
            }
            b->ev.push_back(e);
        }
        b->schedule = 1;
    }
    return WAVE_OK;
}

int wave_batch_info(const wave_batch *b, int32_t *groups, int64_t *workgroups_per_step,
                    int64_t *points_per_step)
{
    if (!b)
        return WAVE_EINVAL;
    if (groups)
        *groups = int32_t(b->groups.size());
    if (workgroups_per_step)
        *workgroups_per_step = b->workgroups;
    if (points_per_step)
        *points_per_step = b->points;
    return WAVE_OK;
}

int wave_batch_sync(wave_batch *b)
{
    if (!b)
        return WAVE_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess || hipGetLastError() != hipSuccess)
        return bfail(b, WAVE_EHIP, "batched run failed");
    if (b->schedule == 2)
        for (const auto &g : b->groups) {
            int flag = 0;
            if (!g.plan.abort || hipMemcpy(&flag, g.plan.abort, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
                return bfail(b, WAVE_EHIP, "schedule 2 status could not be read");
            if (flag)
                return bfail(b, WAVE_EHIP, "schedule 2: a dependency wait gave up; the run's results are invalid");
        }
    if (b->schedule == 3)
        for (const auto &g : b->groups) {
            int flag = 0;
            if (hipMemcpy(&flag, g.items.counters + 18, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
                return bfail(b, WAVE_EHIP, "schedule 3 status could not be read");
            if (flag)
                return bfail(b, WAVE_EHIP, "schedule 3: a barrier wait ran past its limit; the run's results are invalid");
        }
    return WAVE_OK;
}

int wave_batch_set_wait_limit(wave_batch *b, int32_t polls)
{
    if (!b)
        return WAVE_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, WAVE_EHIP, "stream synchronisation failed");
    drop_batch_graph(b);  // the limit is a launch argument of the captured graph
    b->wait_limit = polls;
    return WAVE_OK;
}

int wave_batch_destroy(wave_batch *b)
{
    if (!b)
        return WAVE_OK;
    batch_free(b);
    delete b;
    return WAVE_OK;
}

const char *wave_batch_last_error(const wave_batch *b)
{
    return b ? b->err.c_str() : "";
}

const char *wave_strerror(int code)
{
    switch (code) {
    case WAVE_OK: return "ok";
    case WAVE_EINVAL: return "invalid argument";
    case WAVE_EUNSTABLE: return "time step violates the leapfrog stability limit";
    case WAVE_ESTATE: return "invalid state";
    case WAVE_ENOMEM: return "out of memory";
    case WAVE_EHIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

const char *wave_last_error(const wave_ctx *ctx)
{
    if (!ctx)
        return "";
    return ctx->err.c_str();
}

}  // extern "C"
