// launch.h -- host-side launchers of the SDMD kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "sdmd_dev.h"

namespace sdmd {

// particles phase (one workgroup per push item = (run, patch))
// px: exact square/cubic patch edge of a compiled fast path (0 = sizes read
// from the run descriptor); pc: LDS sizing class 8 / 16 / 32
hipError_t launch_push(int dims, bool split, int px, int pc, bool det, const RunDev *runs, const int2 *items,
                       int n_items, int par, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// transfer (i) + current filter + Maxwell: items (run, region, tile,
// first-item-of-run flag); tx: x extent of the tile, from
// yee_tile_x(dims, region width, filter on); filt: runs with filter passes
int yee_tile_x(int dims, int rs0, bool filt);
void yee_tile_shape(int dims, int tx, int shape[3]);
hipError_t launch_yee(int dims, bool split, int tx, bool filt, bool det, const RunDev *runs, const int4 *items,
                      int n_items, int par, hipStream_t s);

// spectral (PSATD) field phase of one run: pack, transforms, exact k-space
// step, inverse transforms, unpack into the other E/B buffer (the field
// kernel has already written J)
hipError_t launch_spectral(const RunDev *runs, int run, int dims, const int n[3], int par, hipStream_t s);
// the spectral solver's twiddle tables (RunDev::spec_tw), once at set-up
hipError_t launch_spec_twiddles(double2 *tw, hipStream_t s);

// ghost synchronisation of the new fields + insertion of the leavers:
// items (run, kind, a, b); kind 0 ghost chunk starting at a, kind 1 insert
// block a of b
hipError_t launch_post(int dims, bool split, const RunDev *runs, const int4 *items, int n_items, int par_new,
                       hipStream_t s);

// ghost synchronisation alone, components [c0, c0 + nc) of one run
hipError_t launch_ghosts(const RunDev *runs, int run, int total_ghosts, int c0, int nc, hipStream_t s);

// initial fields: global FP64 staging (3 components) -> region interiors of
// components [c0, c0+3)
hipError_t launch_scatter_fields(const RunDev *runs, int run, int ncell, const double *src, int c0, hipStream_t s);
// region interiors of component c -> global FP64 array
hipError_t launch_assemble(const RunDev *runs, int run, int ncell, int comp, double *dst, hipStream_t s);
// Bm = B, then B -= dt/2 curl E on every region interior (buffer par)
hipError_t launch_half_faraday(const RunDev *runs, int run, int ncell, int par, hipStream_t s);

// particles: FP64 staging -> spill store with patch ids
hipError_t launch_convert(int dims, bool split, const RunDev *runs, int run, int n, const double *x, const double *y,
                          const double *z, const double *ux, const double *uy, const double *uz, const double *w,
                          const uint32_t *id, hipStream_t s);
// re-layout of the patch stores of the runs listed in slots[0..n_slots)
// (tally / count parked / plan / move / commit); force = 1 re-lays out even
// without parked particles; count_gx workgroups per run count the parked
// particles
hipError_t launch_relayout(int dims, bool split, RunDev *runs, const int *slots, int n_slots, int count_gx,
                           int move_gx, int commit_gx, int force, hipStream_t s);
// export: live particles -> FP64 arrays at per-segment offsets (off[nseg]
// = start of the spill part)
hipError_t launch_export(int dims, bool split, const RunDev *runs, int run, int seg_max, int nspill, const int *off,
                         double *x, double *y, double *z, double *ux, double *uy, double *uz, double *w, uint32_t *id,
                         int *patch, hipStream_t s);
// diagnostics: partial sums (field energy per block; kinetic per patch)
hipError_t launch_field_energy(const RunDev *runs, int run, int ncell, int par, double *partial, int nblocks,
                               hipStream_t s);
// Gauss-law residual g = div_h E (buffer par) - rho per node, and per-block
// maxima of |g - g0| and |rho| (2 doubles per block)
hipError_t launch_gauss(const RunDev *runs, int run, int ncell, int par, const double *rho, double *g, hipStream_t s);
hipError_t launch_gauss_max(int ncell, const double *g, const double *g0, const double *rho, double *partial,
                            int nblocks, hipStream_t s);
hipError_t launch_kinetic(int dims, bool split, const RunDev *runs, int run, int seg_max, int nspill, double *partial,
                          hipStream_t s);
// charge density (electrons) at primal nodes, global FP64 array (zeroed
// here); det: summed in 64-bit fixed point, then converted in place
hipError_t launch_rho(int dims, bool split, bool det, const RunDev *runs, int run, int seg_max, int nspill, int ncell,
                      double *rho, hipStream_t s);
// a short wait on the device that holds the stream while the host enqueues
hipError_t launch_gate(int us, hipStream_t s);

}  // namespace sdmd
