// Types and constants shared by the host code of libwave.so (wave.hip) and
// its kernel translation units (k_*.hip); the kernels are declared in
// wave_kernels.h.
#pragma once

#include <hip/hip_runtime.h>

#include "wave.h"

namespace wavek {


constexpr int kGhost = 4;
constexpr int kRowAlignBytes = 128;  // interior rows start on this boundary

// 8th-order central second-derivative weights (four points each way).
constexpr double kC0 = -205.0 / 72.0;
constexpr double kCm[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
// max over wavenumbers of |c0 + 2 sum c_m cos(m kh)|, reached at kh = pi;
// it also equals |c0| + 2 sum |c_m|, which bounds |lap u| by this times
// max|u| sum 1/h^2.
constexpr double kSymbolMax = 2048.0 / 315.0;

// largest scaled magnitude a 16-bit field is written with (2^14)
constexpr int kScaledTopExp = 14;

constexpr int elem_bytes(int dtype) { return dtype == WAVE_F32 ? 4 : 2; }
constexpr int kNumKinds = 5;  // storage types WAVE_F32 .. WAVE_BF16_UV
constexpr bool is_uv(int dtype) { return dtype == WAVE_F16_UV || dtype == WAVE_BF16_UV; }

struct alignas(16) f4 {
    float v[4];
};

struct Coefs {
    float ctr;    // c0 * (1/dx^2 + 1/dy^2 + 1/dz^2): the centre counted once
    float cx[4];  // c_m / dx^2
    float cy[4];
    float cz[4];
};

struct StepArgs {
    const void *k;
    const void *cur;
    void *nxt;  // u^{n-1} (adjoint: phi^{m+2}; imaging: phi^m)
    const float *__restrict__ gx;
    const float *__restrict__ gy;
    const float *__restrict__ gz;
    Coefs c;
    int nx, ny, nz;
    int px;             // row pitch in elements
    int x0;             // element offset of interior x = 0 in a row
    long long plane;    // elements per plane
    int nxq;            // ceil(nx / 4): 4-cell columns holding interior cells
    int ntx, nty, nchunks, zc, nwg;
    int src_z, src_y, src_x;  // src_z < 0: no source
    const float *src_ptr;     // device value of this step, or NULL
    float src_val;            // used when src_ptr is NULL
    const int *rec_start;     // [nwg + 1] receiver ranges per work-group
    const long long *rec_off; // element offset of each receiver
    const int *rec_idx;       // receiver number
    float *trace_row;         // row of this step, or NULL
    // 16-bit storage only
    int step;                 // n: this launch writes u^{n+1}
    float k_scale;            // k = stored k * k_scale
    int *exps;                // [4] exponent of u^m in slot m & 3
    unsigned *maxes;          // [4] max |u^m| (float bits) in slot m & 3
    // output field: == nxt for the in-place step (each cell is read, then
    // written, by the same thread), a separate level otherwise
    void *out;
    // imaging: FP64 accumulator in the field layout (8-byte cells)
    double *grad;
    // fused adjoint step: the forward level whose Laplacian the imaging term needs
    const void *aux;
    // u-and-change storage: d^n on entry, d^{n+1} on exit (same cells, same thread)
    void *dlt;
    // z-march direction of the tiled kernels: 0 up, 1 down.  Consecutive
    // launches alternate, so that a launch starts on the planes the one
    // before touched last, which the GPU's memory-side cache still holds.
    // The results do not depend on it: the z taps enter only as the
    // commutative sums u[z+m] + u[z-m].
    int zdown;
};

// What a tiled launch computes (FP32 storage only for the last two):
//   kFwd  u^{n+1} = G (2 u^n - G u^{n-1} + k lap u^n) (+ source, receivers);
//   kAdj  the adjoint step phi^m = 2 psi + k lap psi - G^2 phi^{m+2} with
//         psi = G phi^{m+1} (G applied to every loaded value);
//   kImg  grad += (G phi / k) lap a: the imaging term of one adjoint step;
//   kFus  kAdj from phi^m, phi^{m+1} together with the kImg term of phi^m
//         and a = aux (the same arithmetic, bit for bit, in one pass).
constexpr int kFwd = 0;
constexpr int kAdj = 1;
constexpr int kImg = 2;
constexpr int kFus = 3;

// A shot of a batched run.  `a` holds the shot's arguments with the buffer
// roles of the run's first step (cur = u^{n0}, nxt = u^{n0-1}); step j of
// the run swaps them when j is odd and offsets the trace row and source.
struct ShotDesc {
    StepArgs a;
    float *traces;     // trace buffer base (row n at traces + n * nrec), or NULL
    int nrec;
    int n0;            // step counter at the start of the run
    const float *src;  // source values of the run's steps, or NULL (then no source)
};

// Work items of a batched step: (shot, tile and z-chunk of that shot),
// split into 8 contiguous ranges of about equal work, one per XCD.
struct BatchItems {
    const int *shot;       // [items] shot (index into the group's descriptors)
    const int *lid;        // [items] tile/chunk number within the shot
    const int *xcd_start;  // [9] item range of each XCD
    int *counters;         // [2][8] tickets of the current and the next step
};

// Single-launch run of a batch (schedule 3): the grid barrier between steps
// and its bound.  count, gen and abort are zero at launch.
struct RunSync {
    unsigned *count;             // work-groups arrived at the current barrier
    unsigned *gen;               // barriers opened so far
    int *abort;                  // raised when a barrier wait runs past the limit
    unsigned long long timeout;  // wall-clock ticks a work-group may wait in all
    int j0;                      // step of the run at which this launch starts
    int nsteps;                  // steps of this launch
};

// Data-flow schedule: one launch runs every step of a group of shots.  Each
// shot is pinned to one XCD; an item is (step, shot, tile, z-chunk).
struct FlowShot {
    int desc;            // index into the group's descriptors
    int items;           // tiles x chunks of the shot
    int base;            // first item of the shot within its XCD's items of one step
    int done;            // first completion counter of the shot
    int ntx, nty, nch;   // tiles in x, in y, and z-chunks
    int zreach;          // chunks on each side a chunk's 4-plane halo reaches
};

struct FlowPlan {
    const FlowShot *shots;  // grouped by XCD
    const int *xcd_shot;    // [9] FlowShot range of each XCD
    const int *xcd_items;   // [8] items of one step on each XCD
    int *tickets;           // [8] next ticket of each XCD (zero at launch)
    int *done;              // [items of all shots] steps completed (zero at launch)
    int *abort;             // [1] raised when a wait gives up (zero at launch)
    int nsteps;             // steps of this launch
    int j0;                 // step of the run at which this launch starts
    int wait_limit;         // polls before a wait gives up; < 0: every wait of a step after the first gives up
};

// Tile shapes (float4 columns x thread rows x rows per thread) of the tiled
// kernels, in the order of the variant table.
#define WAVE_TILE_SHAPES(X)                                                                       \
    X(16, 16, 1) X(32, 8, 1) X(32, 8, 2) X(16, 16, 2) X(32, 16, 1) X(64, 4, 2) X(16, 8, 2)       \
    X(32, 8, 4) X(64, 8, 1) X(16, 32, 1) X(32, 16, 2) X(64, 8, 2)

}  // namespace wavek
