// pf_kernels_common.h -- indexing helpers shared by the sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_device.h"

namespace pfk {

// Grid geometry with the boundary rules of the model: periodic in x and y,
// zero-gradient mirror of one ghost layer in z (Sec. 2.1 boundary handling,
// applied here by index arithmetic instead of ghost cells).  With a
// Dirichlet top, plane nz is a stored ghost plane (liquid at a fixed mu):
// nzr = nz + 1 planes can be read and the face above plane nz-1 exists.
struct Geo {
  int nx, ny, nz, nzr, pitch;
  int64_t plane;
  __device__ __forceinline__ int xp(int x) const { return x + 1 == nx ? 0 : x + 1; }
  __device__ __forceinline__ int xm(int x) const { return x == 0 ? nx - 1 : x - 1; }
  __device__ __forceinline__ int yp(int y) const { return y + 1 == ny ? 0 : y + 1; }
  __device__ __forceinline__ int ym(int y) const { return y == 0 ? ny - 1 : y - 1; }
  __device__ __forceinline__ int zp(int z) const { return z + 1 >= nzr ? nzr - 1 : z + 1; }
  __device__ __forceinline__ int zm(int z) const { return z <= 0 ? 0 : z - 1; }
  // plane p with one mirrored ghost plane on each side: -1 -> 0, nz -> nz-1
  // (planes further out are clamped too; they are loaded but never used)
  __device__ __forceinline__ int zc(int p) const { return p < 0 ? 0 : (p >= nzr ? nzr - 1 : p); }
  // a z face lies above plane k (faces on the mirror boundaries carry no flux)
  __device__ __forceinline__ bool zface(int k) const { return k >= 0 && k < nzr - 1; }
  __device__ __forceinline__ int64_t at(int x, int y, int z) const {
    return (int64_t)z * plane + (int64_t)y * pitch + x;
  }
};

template <typename DD>
__device__ __forceinline__ Geo make_geo(const DD& d) {
  Geo g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.nzr = d.nz + (d.top_bc ? 1 : 0);
  g.pitch = d.pitch;
  g.plane = d.plane;
  return g;
}

// Domain owning flattened work item `item` (binary search of the prefix sums).
__device__ __forceinline__ int find_domain(const int32_t* first_g, int ndom, int item) {
  const PF_CONST int32_t* first = to_const(first_g);
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One work item: an x-y tile of tx * ty columns and a chunk of zc planes.
struct WorkTile {
  int x0, y0;    // tile origin
  int lx, ly;    // this thread's column inside the tile
  int x, y;      // this thread's column in the domain
  int z0, z1;    // planes [z0, z1)
  bool item_ok;  // the block has an item (false for padding blocks)
  bool valid;    // item present and column inside the domain
};

constexpr int kXcds = 8;

// Block lb (relative to the domain's first block, a multiple of 8) -> tile.
// Work groups are dispatched round-robin over the 8 XCDs, each with its own
// L2, so block lb runs on XCD lb % 8.  In y-slab order (xmode = 1) XCD j
// owns tile rows [j rs, (j+1) rs) over the whole height and walks them x
// fastest, then y, then z: tiles that read each other's halo cells share one
// L2, and every XCD gets the same share of the costly interface planes.
// Plain order (xmode = 0) is x fastest, then y, then z chunk.  Both orders
// leave padding blocks without an item.
template <typename DD>
__device__ __forceinline__ WorkTile decode_item(const DD& d, int lb, int tid) {
  WorkTile w;
  int ix = 0, iy = 0, iz = 0;
  bool ok;
  if (d.xmode) {
    const int j = lb % kXcds, p = lb / kXcds;
    const int y_lo = j * d.rs;
    const int rows = min(d.rs, d.nty - y_lo);
    ok = rows > 0;
    if (ok) {
      const int per_z = rows * d.ntx;
      iz = p / per_z;
      const int rem = p - iz * per_z;
      iy = y_lo + rem / d.ntx;
      ix = rem % d.ntx;
      ok = iz < d.nzc;
    }
  } else {
    ix = lb % d.ntx;
    const int r = lb / d.ntx;
    iy = r % d.nty;
    iz = r / d.nty;
    ok = iz < d.nzc;
  }
  if (!ok) iz = d.nzc;  // empty plane range
  w.item_ok = ok;
  w.lx = tid % d.tx;
  w.ly = tid / d.tx;
  w.x0 = ix * d.tx;
  w.y0 = iy * d.ty;
  w.x = w.x0 + w.lx;
  w.y = w.y0 + w.ly;
  w.z0 = iz * d.zc;
  w.z1 = min(d.nz, w.z0 + d.zc);
  w.valid = ok && w.x < d.nx && w.y < d.ny;
  return w;
}

// Descriptor of domain di through the constant address space.
__device__ __forceinline__ const PF_CONST DevDomain& domain_at(DevDomain* const* doms, int di) {
  return *to_const(to_const(doms)[di]);
}
__device__ __forceinline__ int first_item(const int32_t* first, int di) {
  return to_const(first)[di];
}

hipError_t launch_phi_tiled(const struct LaunchSet& L, int prec, bool aniso, hipStream_t s);
hipError_t launch_mu_tiled(const struct LaunchSet& L, int prec, hipStream_t s);

}  // namespace pfk
