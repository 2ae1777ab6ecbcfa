// pf_io.hip -- the output path outside the time step (Sec. 3.2, Input/
// Output): FP32 checkpoints of the state, and one triangle mesh per phase of
// its interfaces from a marching-cubes pass over phi (after Lorensen and
// Cline).
//
// Checkpoints: a pack kernel rounds the six fields of the current copy to
// float into a contiguous [f][z][y][x] block (written into the other copy,
// which holds nothing between steps); the host writes that block to the
// file.  Loading reverses it.
//
// Meshes: one thread per cube of eight neighbouring cell centres (periodic
// in x and y, open at the first and last z planes), one work group per row
// of cubes.  Corner c of the cube at
// (x, y, z) is the cell (x + (c & 1), y + (c >> 1 & 1), z + (c >> 2 & 1));
// it is inside when phi_a > iso.  The triangles of each of the 256 inside
// patterns come from a table built at compile time by this rule: on each
// cube face (corners counter-clockwise seen from outside) every run of
// consecutive inside corners is cut off by a segment from the crossing that
// leaves the run to the crossing that enters it; the segments close into
// loops, and each loop, started at its lowest-numbered edge, is split into
// a fan wound so that normals point out of the phase.  A vertex on the edge
// from corner A to corner B (A the lower) sits at A + t (B - A) with
// t = (iso - phi_A) / (phi_B - phi_A) in FP64, stored as float.  Triangles
// are reserved per wave with one atomic add, so their order is not fixed.
#include <hip/hip_runtime.h>

#include "pf_device.h"
#include "pf_launch.h"

namespace pfk {

// ------------------------------------------------------------- checkpoint

template <typename R>
__global__ __launch_bounds__(256) void ckpt_pack_kernel(const DevDomain* dom, int src, float* out) {
  const DevDomain& d = *dom;
  const R* base = static_cast<const R*>(d.copy[src]);
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c % d.nx, r = c / d.nx;
    const int64_t o = (r / d.ny) * d.plane + (r % d.ny) * d.pitch + x;
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) out[f * cells + c] = (float)base[f * d.fstride + o];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void ckpt_unpack_kernel(const DevDomain* dom, int dst,
                                                          const float* in) {
  const DevDomain& d = *dom;
  R* base = static_cast<R*>(d.copy[dst]);
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c % d.nx, r = c / d.nx;
    const int64_t o = (r / d.ny) * d.plane + (r % d.ny) * d.pitch + x;
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) base[f * d.fstride + o] = (R)in[f * cells + c];
  }
}

// One field of a copy as dense FP64 [z][y][x] (host readback), and back
// (host initialisation, rounded to the domain's precision).
template <typename R>
__global__ __launch_bounds__(256) void field_pack_kernel(const DevDomain* dom, int src, int f,
                                                         double* out) {
  const DevDomain& d = *dom;
  const R* base = static_cast<const R*>(d.copy[src]) + f * d.fstride;
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c % d.nx, r = c / d.nx;
    out[c] = (double)base[(r / d.ny) * d.plane + (r % d.ny) * d.pitch + x];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void field_unpack_kernel(const DevDomain* dom, int dst, int f,
                                                           const double* in) {
  const DevDomain& d = *dom;
  R* base = static_cast<R*>(d.copy[dst]) + f * d.fstride;
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c % d.nx, r = c / d.nx;
    base[(r / d.ny) * d.plane + (r % d.ny) * d.pitch + x] = (R)in[c];
  }
}

namespace {
int grid_for(int64_t items) {
  const int64_t b = (items + 255) / 256;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}
}  // namespace

hipError_t launch_ckpt_pack(const DevDomain* dom, int prec, int64_t cells, int src, float* out,
                            hipStream_t s) {
  if (prec == 0)
    ckpt_pack_kernel<double><<<grid_for(cells), 256, 0, s>>>(dom, src, out);
  else
    ckpt_pack_kernel<float><<<grid_for(cells), 256, 0, s>>>(dom, src, out);
  return hipGetLastError();
}

hipError_t launch_ckpt_unpack(const DevDomain* dom, int prec, int64_t cells, int dst,
                              const float* in, hipStream_t s) {
  if (prec == 0)
    ckpt_unpack_kernel<double><<<grid_for(cells), 256, 0, s>>>(dom, dst, in);
  else
    ckpt_unpack_kernel<float><<<grid_for(cells), 256, 0, s>>>(dom, dst, in);
  return hipGetLastError();
}

hipError_t launch_field_pack(const DevDomain* dom, int prec, int64_t cells, int src, int f,
                             double* out, hipStream_t s) {
  if (prec == 0)
    field_pack_kernel<double><<<grid_for(cells), 256, 0, s>>>(dom, src, f, out);
  else
    field_pack_kernel<float><<<grid_for(cells), 256, 0, s>>>(dom, src, f, out);
  return hipGetLastError();
}

hipError_t launch_field_unpack(const DevDomain* dom, int prec, int64_t cells, int dst, int f,
                               const double* in, hipStream_t s) {
  if (prec == 0)
    field_unpack_kernel<double><<<grid_for(cells), 256, 0, s>>>(dom, dst, f, in);
  else
    field_unpack_kernel<float><<<grid_for(cells), 256, 0, s>>>(dom, dst, f, in);
  return hipGetLastError();
}

// ------------------------------------------------------- marching cubes

constexpr int kMcMaxTri = 5;  // the most any of the 256 cases needs

// The twelve cube edges as corner pairs (lower corner first): x edges, then
// y edges, then z edges, each group ordered by the other two coordinates.
constexpr int kEdge[12][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3},
                              {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
// Faces -x, +x, -y, +y, -z, +z: corners counter-clockwise seen from outside.
constexpr int kFaceCorner[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                   {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};

struct McCase {
  int8_t n;                   // triangles
  int8_t e[3 * kMcMaxTri];    // their edges, three per triangle
};
struct McTable {
  McCase c[256];
};

constexpr int edge_between(int a, int b) {
  for (int e = 0; e < 12; ++e)
    if ((kEdge[e][0] == a && kEdge[e][1] == b) || (kEdge[e][0] == b && kEdge[e][1] == a)) return e;
  return -1;
}

constexpr McCase make_case(int mask) {
  McCase r{};
  // successor of each crossed edge along the loops; -1: not crossed
  int succ[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  for (int f = 0; f < 6; ++f) {
    bool in[4] = {};
    int edge[4] = {};  // edge[i]: between face corners i and i+1
    for (int i = 0; i < 4; ++i) {
      in[i] = (mask >> kFaceCorner[f][i]) & 1;
      edge[i] = edge_between(kFaceCorner[f][i], kFaceCorner[f][(i + 1) & 3]);
    }
    // a crossing that leaves a run (inside at i, outside at i+1) links to
    // the crossing that entered it (outside before the run's first corner)
    for (int i = 0; i < 4; ++i) {
      if (!in[i] || in[(i + 1) & 3]) continue;
      int k = i;
      while (in[(k + 3) & 3]) k = (k + 3) & 3;
      succ[edge[i]] = edge[(k + 3) & 3];
    }
  }
  bool seen[12] = {};
  for (int s = 0; s < 12; ++s) {
    if (succ[s] < 0 || seen[s]) continue;
    int loop[12] = {};
    int m = 0;
    for (int e = s; !seen[e]; e = succ[e]) {
      seen[e] = true;
      loop[m++] = e;
    }
    for (int i = 1; i + 1 < m; ++i) {
      r.e[3 * r.n + 0] = (int8_t)loop[0];
      r.e[3 * r.n + 1] = (int8_t)loop[i + 1];
      r.e[3 * r.n + 2] = (int8_t)loop[i];
      ++r.n;
    }
  }
  return r;
}

constexpr McTable make_table() {
  McTable t{};
  for (int m = 0; m < 256; ++m) t.c[m] = make_case(m);
  return t;
}

__constant__ McTable kMc = make_table();

// One work group per row of cubes (fixed y and z), threads along x, so that
// neighbouring lanes share corner rows and no 64-bit division is needed.
template <typename R>
__global__ __launch_bounds__(256) void mesh_kernel(const DevDomain* dom, int phase, double iso,
                                                   float* out, int64_t cap,
                                                   unsigned long long* count) {
  const DevDomain& d = *dom;
  const R* f = static_cast<const R*>(d.copy[d.parity]) + (int64_t)phase * d.fstride;
  const int nx = d.nx, ny = d.ny;
  const int rows = ny * (d.nz - 1);
  const int lane = threadIdx.x & 63;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = row % ny, z = row / ny;
    const int64_t ys[2] = {(int64_t)y * d.pitch, (int64_t)(y + 1 == ny ? 0 : y + 1) * d.pitch};
    const int64_t zs[2] = {(int64_t)z * d.plane, (int64_t)(z + 1) * d.plane};
    for (int x0 = 0; x0 < nx; x0 += blockDim.x) {  // same trip count for the whole group
      const int x = x0 + (int)threadIdx.x;
      double v[8];
      int mask = 0;
      if (x < nx) {
        const int xs[2] = {x, x + 1 == nx ? 0 : x + 1};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          v[k] = (double)f[zs[k >> 2] + ys[(k >> 1) & 1] + xs[k & 1]];
          mask |= (v[k] > iso ? 1 : 0) << k;
        }
      }
      // most waves cross no surface: leave before the table and the scan
      if (__ballot(mask != 0 && mask != 255) == 0) continue;
      const int n = kMc.c[mask].n;  // 0 for masks 0 and 255, and for idle lanes
      // exclusive prefix of n over the wave, one atomic add per wave
      int pre = n;
#pragma unroll
      for (int s = 1; s < 64; s <<= 1) {
        const int o = __shfl_up(pre, s, 64);
        if (lane >= s) pre += o;
      }
      const int total = __shfl(pre, 63, 64);
      if (total == 0) continue;  // uniform over the wave
      pre -= n;
      unsigned long long base = 0;
      if (lane == 63) base = atomicAdd(count, (unsigned long long)total);
      base = __shfl(base, 63, 64);
      for (int t = 0; t < n; ++t) {
        const int64_t slot = (int64_t)base + pre + t;
        if (slot >= cap) break;
        float* o = out + 9 * slot;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int e = kMc.c[mask].e[3 * t + q];
          const int a = kEdge[e][0], b = kEdge[e][1];
          const double tt = (iso - v[a]) / (v[b] - v[a]);
          const int axis = e >> 2;
          const double p[3] = {(double)(x + (a & 1)), (double)(y + ((a >> 1) & 1)),
                               (double)(z + ((a >> 2) & 1))};
          o[3 * q + 0] = (float)(axis == 0 ? p[0] + tt : p[0]);
          o[3 * q + 1] = (float)(axis == 1 ? p[1] + tt : p[1]);
          o[3 * q + 2] = (float)(axis == 2 ? p[2] + tt : p[2]);
        }
      }
    }
  }
}

hipError_t launch_mesh(const DevDomain* dom, int prec, int64_t rows, int phase, double iso,
                       float* out, int64_t cap, unsigned long long* count, hipStream_t s) {
  const int grid = (int)(rows < 16384 ? (rows > 0 ? rows : 1) : 16384);
  if (prec == 0)
    mesh_kernel<double><<<grid, 256, 0, s>>>(dom, phase, iso, out, cap, count);
  else
    mesh_kernel<float><<<grid, 256, 0, s>>>(dom, phase, iso, out, cap, count);
  return hipGetLastError();
}

}  // namespace pfk
