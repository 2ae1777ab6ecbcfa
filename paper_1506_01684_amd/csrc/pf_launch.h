// pf_launch.h -- host-side launch wrappers of the phase-field kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_device.h"

namespace pfk {

// A launch covers `ndom` domains whose descriptors live in device memory at
// `doms`; `first` (device, ndom+1 entries) is the prefix sum of work items
// (x-y tiles times z chunks) per domain, `total` its last entry.
struct LaunchSet {
  DevDomain* const* doms;  // device array of descriptor pointers
  const int32_t* first;
  int32_t ndom;
  int32_t total;
  // one domain: its per-item words (the sweeps' classification), so that a
  // work group can test its item with one load; a pack: null
  const uint32_t* words;
};

// Threads per work group of the sweeps (tile tx * ty).
constexpr int kTileThreads = 256;
constexpr int kTileWaves = kTileThreads / 64;
// Most z planes per work item of the tiled sweeps.
constexpr int kMaxZc = 32;

// The step's prologue: prologue_kernel (one work group per domain: copy
// choice, window decision, counters, step counter), then coef_kernel
// (kCoefBlocks work groups of kCoefThreads per domain: the per-plane
// coefficient table).
constexpr int kCoefBlocks = 16, kCoefThreads = 128;
hipError_t launch_prologue(const LaunchSet& L, int prec, hipStream_t s);
hipError_t launch_window(const LaunchSet& L, int prec, hipStream_t s);
hipError_t launch_ghost(const DevDomain* dom, int prec, int nx, int ny, hipStream_t s);
hipError_t launch_phi(const LaunchSet& L, int prec, bool aniso, int variant, hipStream_t s);
hipError_t launch_mu(const LaunchSet& L, int prec, int variant, hipStream_t s);

// Fill the current state copy: column phase map (int8, nx*ny) below
// solid_height, liquid above, uniform mu.
hipError_t launch_fill(const DevDomain* dom, int prec, int nx, int ny, int nz,
                       const int8_t* phase_map, int32_t solid_height, double mu0, double mu1,
                       hipStream_t s);

// Diagnostics of the state in copy `parity` at time t (t < 0: the time
// of the device step counter): out[0..9] =
// sum_c0, sum_c1, sum_phi0..3, max |sum phi - 1|, min phi, max phi,
// non-finite cell count.  `partials` holds kDiagBlocks * 10 doubles.
constexpr int kDiagBlocks = 480;
constexpr int kDiagValues = 10;
hipError_t launch_diag(const DevDomain* dom, int prec, int nx, int ny, int nz, double t,
                       double* partials, double* out, hipStream_t s);
// The same diagnostics of six fields the caller holds: field f of cell
// (x,y,z) at base[f fstride + z plane + y pitch + x] (elements of the
// precision), with the temperature and concentration coefficients given
// here instead of a domain's descriptor.
struct DiagView {
  const void* base;
  int32_t nx, ny, nz;
  int64_t pitch, plane, fstride;
  double T0, G, dx, zoff, v, TE;
  int64_t shifts;
  double chi0[NP][NM], chi1[NP][NM], c0[NP][NM], c1[NP][NM];
};
hipError_t launch_diag_view(const DiagView& view, int prec, double t, double* partials,
                            double* out, hipStream_t s);

// Output path (pf_io.hip).  Checkpoints: the six fields of copy `src`
// rounded to float into out[f][z][y][x] (cells = nx ny nz), and back into
// copy `dst`.  Meshes: marching cubes of phi_phase = iso over the current
// copy, rows = ny (nz - 1) rows of cubes; triangles (9 floats each) go to
// out[0 .. cap), *count (device, zeroed by the caller) receives the total.
hipError_t launch_ckpt_pack(const DevDomain* dom, int prec, int64_t cells, int src, float* out,
                            hipStream_t s);
hipError_t launch_ckpt_unpack(const DevDomain* dom, int prec, int64_t cells, int dst,
                              const float* in, hipStream_t s);
// Clear the both-copies mark of n chunk flags of the current copy, after
// the other copy has served as host staging.
hipError_t launch_drop_same(uint8_t* flags, int64_t n, hipStream_t s);
// Host boundary: field f of copy `src` as dense FP64 out[z][y][x], and
// dense FP64 in[z][y][x] rounded into field f of copy `dst`.
hipError_t launch_field_pack(const DevDomain* dom, int prec, int64_t cells, int src, int f,
                             double* out, hipStream_t s);
hipError_t launch_field_unpack(const DevDomain* dom, int prec, int64_t cells, int dst, int f,
                               const double* in, hipStream_t s);
hipError_t launch_mesh(const DevDomain* dom, int prec, int64_t rows, int phase, double iso,
                       float* out, int64_t cap, unsigned long long* count, hipStream_t s);

}  // namespace pfk
