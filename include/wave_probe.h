/*
 * wave_probe.h -- bandwidth probes shipped beside libwave.so (libwave_probe.so).
 *
 * Not part of the propagator: plain streaming kernels of known traffic,
 * used to measure the HBM bandwidth this GPU actually sustains for the
 * propagator's access pattern and to calibrate hardware byte counters, and
 * the cost of synchronising work-groups inside one launch against that of
 * a launch.
 * All pointers are device pointers of n floats (16-byte aligned, n a
 * multiple of 4); work is enqueued on `stream` and not waited for.
 * Return 0, or -1 for bad arguments / -5 for a failed launch.
 */
#ifndef WAVE_PROBE_H
#define WAVE_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[i] = src[i]: 8 bytes of HBM traffic per element. */
int probe_copy(const float *src, float *dst, int64_t n, void *stream);

/* d[i] = a[i] + b[i] + c[i]: three reads and one write per element (16 bytes),
 * the access mix of one propagator update. */
int probe_read3_write1(const float *a, const float *b, const float *c, float *d, int64_t n,
                       void *stream);

/* o[i] = a[i] + b[i] + c[i] + d[i]; g[i] += o[i] in FP64 (g: n doubles):
 * four FP32 reads, an FP64 read and write and an FP32 write per element
 * (36 bytes), the access mix of one fused adjoint-and-imaging update. */
int probe_adjoint_mix(const float *a, const float *b, const float *c, const float *d, double *g,
                      float *o, int64_t n, void *stream);

/* Synchronisation cost inside one cooperative launch of `blocks` (>= 2)
 * work-groups of 256 threads: nsteps grid-wide barriers (ring = 0) or waits
 * for the two ring neighbours' step counters (ring != 0), each work-group
 * arriving with an agent-scope release and leaving after an agent-scope
 * acquire, as the library's single-launch batch does between steps.
 * words: device ints, at least 4 + blocks, all zero on entry; words[2] is
 * raised (and the launch ends) if a wait passes timeout_s seconds of wall
 * clock.  -1 for bad arguments or a device without cooperative launches,
 * -5 if the launch fails (for instance more work-groups than fit at once). */
int probe_sync(int *words, int blocks, int nsteps, int ring, double timeout_s, void *stream);

/* An empty kernel of `blocks` work-groups: the cost of a launch. */
int probe_empty(int blocks, void *stream);

/* The propagator step's HBM access pattern without its arithmetic, on three
 * fields in the library's padded layout (nz + 8 planes of ny + 8 rows of
 * `pitch` floats, interior x from float `x0`; 4 ghost planes and rows on
 * each side): tiles of 256 cells x 8 rows and z-chunks of zc planes, each
 * work-group marching its chunk (from the top when `down`), reading a four
 * planes ahead of the march and b, k at the plane, and writing
 * b = a + b + k in place: 16 bytes per interior cell, as one step.
 * Launches that swap a and b and alternate `down` reproduce the library's
 * launch sequence.  -1 for bad arguments (nx and x0 multiples of 4,
 * x0 >= 4, pitch >= x0 + nx + 4). */
int probe_step_stream(const float *a, float *b, const float *k, int nx, int ny, int nz, int64_t pitch,
                      int64_t x0, int zc, int down, void *stream);

/* The same for the 16-bit storage forms: 2-byte cells, fields of nz + 8
 * planes of ny + 8 rows of `pitch` cells with interior x from cell x0 (nx,
 * x0, pitch multiples of 4; 8-byte aligned pointers).  Tiles of 32 x ty
 * threads, each thread 4 cells in ry rows ((ty, ry) one of (8, 1), (8, 2),
 * (16, 1), (16, 2), (32, 1): the 16-bit step kernels' tiles of 128 cells),
 * z-chunks of zc planes.  o == NULL: the two-level step's pattern, u read
 * four planes ahead of the march and p, k at the plane, p = u ^ p ^ k
 * written in place (8 bytes per cell).  o != NULL: the u-and-change step's
 * pattern, u ahead and p (the change), k at the plane, o = u ^ k written to
 * o and p = p ^ u in place (10 bytes per cell).  Cache policies are the
 * step kernels': u (and the change p) read with the default policy, the
 * other accesses non-temporal.  -1 for bad arguments. */
int probe_step_stream16(const void *u, void *p, void *o, const void *k, int nx, int ny, int nz, int64_t pitch,
                        int64_t x0, int zc, int ty, int ry, int down, void *stream);

/* The fused adjoint step's access pattern without its arithmetic, on FP32
 * fields in the layout above (c, a, p, k) and an FP64 accumulator g with the
 * same layout in 8-byte cells (16-byte aligned pointers): c and a read four
 * planes ahead of the march (default policy), p and k at the plane
 * (non-temporal), g read and written at the plane (default policy), and
 * p = c ^ a ^ p ^ k written in place (non-temporal), 36 bytes per cell; the
 * first 16 bytes of a thread's 32 accumulator bytes are XORed with c's 16,
 * the second with a's.  Tiles of 32 x ty threads (ty 8 or 16), each thread
 * 4 cells of one row, z-chunks of zc planes, as the adjoint kernel tiles a
 * grid.  -1 for bad arguments (as probe_step_stream, and the accumulator's
 * plane under 2 GiB). */
int probe_adjoint_stream(const float *c, const float *a, float *p, const float *k, double *g, int nx, int ny,
                         int nz, int64_t pitch, int64_t x0, int zc, int ty, int down, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WAVE_PROBE_H */
