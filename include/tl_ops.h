/*
 * tl_ops.h -- operator-level entry points of the two-level thermal library,
 * on caller-owned device buffers.  These expose the fine-level heat operator
 * on its own (for verification and bandwidth measurement); the simulation
 * API in tl.h uses the same kernels.
 *
 * Device layout ("padded"): a grid of nx x ny x nz Q1 cells has
 * (nx+1) x (ny+1) x (nz+1) nodes stored with one ghost layer on every side,
 * node (i,j,k) at ((k+1)*(ny+3) + (j+1))*px + (i+1), where the row pitch px
 * is nx+3 rounded up to a multiple of 32 (so every row starts on a 128-byte
 * boundary of a 256-byte aligned buffer); ghost and pitch-padding entries
 * are zero.  A per-element quantity of element (i,j,k) is stored at the padded
 * index of its lowest corner node (i,j,k); all other entries are zero.
 */
#ifndef TL_OPS_H
#define TL_OPS_H

#include <stddef.h>
#include "tl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* nx x ny x nz Q1 cells of spacing hx, hy, hz [m]. */
typedef struct {
  int nx, ny, nz;
  double hx, hy, hz;
} tl_grid;

/* Number of entries of a padded array of this grid. */
size_t tl_op_padded_size(const tl_grid* grid);

/* Copy between the plain layout (nodes: i + (nx+1)*(j + (ny+1)*k); elements:
 * i + nx*(j + ny*k)) and the padded layout.  kind 0 = nodal, 1 = per-element;
 * elem_bytes 4 (float) or 8 (double).  pack writes zeros into every padded
 * entry it does not fill.  Both pointers are device pointers. */
tl_status tl_op_pack(const tl_grid* grid, int kind, int elem_bytes,
                     const void* plain, void* padded, void* hip_stream);
tl_status tl_op_unpack(const tl_grid* grid, int kind, int elem_bytes,
                       const void* padded, void* plain, void* hip_stream);

/* Matrix-free Q1 heat operator on every node of the grid:
 *   y_i = d_i v_i + sum_{elements e containing i} kappa_e (K_e v_e)_i
 * with K_e the exact Q1 element stiffness of an hx x hy x hz box (the
 * diffusion term of the paper's thermal model, Section 2.1, discretised
 * with trilinear hexahedra).  d, kappa, v, y are padded device arrays of
 * doubles (precision TL_FP64) or floats (TL_MIXED); y must not overlap the
 * inputs.  kernel: 0 = chosen by grid size (z-marching above 4 Mi nodes with
 * nz >= 8, else tiled), 1 = 3D tiles of 16 x 4 x 4 nodes staged with their
 * halo in LDS, 2 = z-marching columns of 64 x 4 nodes with a sliding
 * register window.  Every kernel sums each node's terms in the same order,
 * so all choices give bitwise-equal y.  blocks: workgroups to launch, 0 for
 * the kernel's own choice, else a positive multiple of 8 up to 2^20 (each
 * workgroup strides over its share of tiles or columns).  `repeat` >= 1
 * launches the operator that many times back to back (for timing).  The
 * call waits for the launches on hip_stream.  Errors: TL_EINVAL for a bad
 * grid, null pointers, repeat < 1, an unknown precision or kernel, or a bad
 * workgroup count; TL_EDEVICE if a HIP call fails. */
tl_status tl_op_apply(const tl_grid* grid, int precision, int kernel,
                      int blocks, const void* d, const void* kappa,
                      const void* v, void* y, int repeat, void* hip_stream);

/* Cost of a device-wide synchronisation between dependent steps on this
 * GPU, for the choice between one launch per step and a persistent kernel
 * that synchronises inside (the batched fine phase of the paper's local
 * problems, Section 4, runs one launch per step).  `rounds` dependent sweeps
 * over the n doubles of `data` (device memory; each entry is mixed with one
 * 4099 entries on, so a sweep reads other workgroups' results of the one
 * before) run on `blocks` workgroups of 256 threads: barrier = 0 launches
 * one kernel per sweep; barrier = 1 runs all sweeps in one cooperative
 * launch with a grid barrier after each (release arrival, bounded relaxed
 * polling, acquire fence).  ctl: >= 1024 bytes of device memory the call
 * zero-fills and uses for the barrier.  *us_out receives the elapsed time
 * of the queued work in microseconds (HIP events on hip_stream).  Errors:
 * TL_EINVAL for null pointers, n < 1, rounds < 1, blocks < 1, or a barrier
 * run with more workgroups than the device holds at once (all must be
 * resident); TL_EDEVICE if a HIP call fails or the barrier's bounded wait
 * ran out. */
tl_status tl_op_sync_probe(int blocks, int rounds, int barrier, double* data,
                           size_t n, void* ctl, double* us_out,
                           void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* TL_OPS_H */
