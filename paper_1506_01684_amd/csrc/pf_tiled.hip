// pf_tiled.hip -- face-sharing z-marching variant of the two sweeps.
//
// A work group of 256 threads owns an x-y tile (64x4 or 32x8 columns; FP64
// always 32x8, whose halo ring is smaller) and
// marches over a chunk of z planes.  The phi^n planes it needs are staged in
// LDS with a one-cell halo ring (one plane for the isotropic phi-sweep,
// a ring of three planes k-1, k, k+1 when tangential face gradients are
// needed: anisotropic phi-sweep and the mu-sweep's anti-trapping current).
// Every face of the tile is evaluated once (Sec. 3.3 buffers staggered
// values so each is computed once; here a z face lives in registers from
// one plane to the next and x/y faces are exchanged through LDS):
//   - each thread evaluates the upper x and y faces of its column and the
//     z face above its cell;
//   - the tile's lower-edge x and y faces are evaluated by the first lanes
//     of one wave, rotating over the planes, through the same code path as
//     all other faces of that direction, so every face rounds identically
//     wherever it is computed;
//   - the next plane's loads are issued before the face stage and written
//     to LDS after it, so their latency overlaps the arithmetic.
// Work items may take cheaper bodies that give bitwise the same result:
//   - phi_bulk_kernel copies (or keeps) the chunks that hold one pure phase
//     at a fixed point with everything around them, before the phi-sweep;
//   - the mu-sweep's items that hold one pure phase before and after the
//     phi-sweep read mu alone (mu_pure_item);
//   - FP64 items whose faces cannot carry the anti-trapping current (no
//     liquid, or only liquid, around them; classified by the phi-sweep)
//     take a lighter body that stages one phi^n plane and no phi^{n+1}
//     neighbours (mu_bulk_item).
// The last two run in one FP64 launch (mu_light_f64) before the full
// kernel, which passes their items over.  A single domain's launch also
// passes the per-item words, so that a work group whose item an earlier
// launch of the step took leaves after one load.
// In the phi-sweep a face enters its two cells' A_a through two shares
// (face_pq): the one for the cell below the face stays in the registers of
// the thread that evaluated it, only the one for the cell above goes
// through LDS, which halves the face buffers.
// LDS layout avoids bank conflicts: phi is stored as 16-byte vectors
// (two doubles or four floats per lane access) and face values as
// structure of arrays (consecutive lanes touch consecutive words).
#include <hip/hip_runtime.h>

#include "pf_device.h"
#include "pf_kernels_common.h"
#include "pf_launch.h"

namespace pfk {

template <typename R>
struct V4 {
  R v[4];
};

// LDS capacities per tile.  FP32 tiles are 64x4 (32x8 when nx < 48); FP64
// tiles are always 32x8.
constexpr int kMaxHalo = 400;  // (tx+2)(ty+2): 66*6 = 396, 34*10 = 340
constexpr int kMaxFx = 264;    // ty (tx+1): 4*65 = 260, 8*33 = 264
template <typename R>
constexpr int kHaloCap = sizeof(R) == 8 ? 340 : kMaxHalo;
template <typename R>
constexpr int kFyCap = sizeof(R) == 8 ? 288 : 320;  // (ty+1) tx: 5*64 = 320, 9*32 = 288

// LDS ring of phi planes: NSLOT planes of (tx+2)(ty+2) cells.
template <typename R, int NSLOT>
struct LdsPhi;

template <int NSLOT>
struct LdsPhi<double, NSLOT> {
  double2 lo[NSLOT][kHaloCap<double>];  // phi_0, phi_1
  double2 hi[NSLOT][kHaloCap<double>];  // phi_2, phi_3
  __device__ __forceinline__ V4<double> get(int s, int c) const {
    const double2 a = lo[s][c], b = hi[s][c];
    return {{a.x, a.y, b.x, b.y}};
  }
  __device__ __forceinline__ void put(int s, int c, const V4<double>& v) {
    lo[s][c] = make_double2(v.v[0], v.v[1]);
    hi[s][c] = make_double2(v.v[2], v.v[3]);
  }
};

template <int NSLOT>
struct LdsPhi<float, NSLOT> {
  float4 q[NSLOT][kMaxHalo];
  __device__ __forceinline__ V4<float> get(int s, int c) const {
    const float4 a = q[s][c];
    return {{a.x, a.y, a.z, a.w}};
  }
  __device__ __forceinline__ void put(int s, int c, const V4<float>& v) {
    q[s][c] = make_float4(v.v[0], v.v[1], v.v[2], v.v[3]);
  }
};

// LDS plane of mu^n (one slot, tile plus halo ring): 16-byte (FP64) or
// 8-byte (FP32) pairs per cell.
template <typename R>
struct LdsMu;
template <>
struct LdsMu<double> {
  double2 m[kHaloCap<double>];
  __device__ __forceinline__ void get(int c, double out[NM]) const {
    const double2 v = m[c];
    out[0] = v.x;
    out[1] = v.y;
  }
  __device__ __forceinline__ void put(int c, const double v[NM]) { m[c] = make_double2(v[0], v[1]); }
};
template <>
struct LdsMu<float> {
  float2 m[kMaxHalo];
  __device__ __forceinline__ void get(int c, float out[NM]) const {
    const float2 v = m[c];
    out[0] = v.x;
    out[1] = v.y;
  }
  __device__ __forceinline__ void put(int c, const float v[NM]) { m[c] = make_float2(v[0], v[1]); }
};

// Per-item geometry of one thread.  In-plane offsets are byte offsets that
// fit 32 bits; plane and field offsets are added to uniform base pointers,
// so loads take the scalar-base + 32-bit vector-offset form.
struct TileGeo {
  int tx, ty, lx, ly, x0, y0, z0, z1;
  bool item_ok, valid;
  int own_c;        // LDS index of the own column
  uint32_t own_b;   // in-plane byte offset of the own column (wrapped for idle threads)
  int halo_c;       // LDS index of the halo cell this thread loads (-1: none)
  uint32_t halo_b;
  __device__ __forceinline__ int ci(int cx, int cy) const { return cy * (tx + 2) + cx; }
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

template <typename R, typename DD>
__device__ __forceinline__ TileGeo make_tile(const DD& d, int local, int t) {
  TileGeo G;
  const WorkTile w = decode_item(d, local, t);
  G.tx = d.tx;
  G.ty = d.ty;
  G.lx = w.lx;
  G.ly = w.ly;
  G.x0 = w.x0;
  G.y0 = w.y0;
  G.z0 = w.z0;
  G.z1 = w.z1;
  G.item_ok = w.item_ok;
  G.valid = w.valid;
  G.own_c = G.ci(w.lx + 1, w.ly + 1);
  const int gx = wrap_mod(w.x, d.nx), gy = wrap_mod(w.y, d.ny);
  G.own_b = (uint32_t)(((int64_t)gy * d.pitch + gx) * (int64_t)sizeof(R));
  const int nhalo = 2 * (G.tx + 2) + 2 * G.ty;
  G.halo_c = -1;
  G.halo_b = 0;
  if (t < nhalo) {
    int cx, cy;
    if (t < G.tx + 2) {
      cx = t;
      cy = 0;
    } else if (t < 2 * (G.tx + 2)) {
      cx = t - (G.tx + 2);
      cy = G.ty + 1;
    } else if (t < 2 * (G.tx + 2) + G.ty) {
      cx = 0;
      cy = t - 2 * (G.tx + 2) + 1;
    } else {
      cx = G.tx + 1;
      cy = t - 2 * (G.tx + 2) - G.ty + 1;
    }
    G.halo_c = G.ci(cx, cy);
    const int hx = wrap_mod(G.x0 - 1 + cx, d.nx), hy = wrap_mod(G.y0 - 1 + cy, d.ny);
    G.halo_b = (uint32_t)(((int64_t)hy * d.pitch + hx) * (int64_t)sizeof(R));
  }
  return G;
}

template <typename R>
__device__ __forceinline__ R ldg(const PF_GLOBAL char* base, uint32_t boff) {
  return *reinterpret_cast<const PF_GLOBAL R*>(base + boff);
}
template <typename R>
__device__ __forceinline__ void stg(PF_GLOBAL char* base, uint32_t boff, R v) {
  *reinterpret_cast<PF_GLOBAL R*>(base + boff) = v;
}

// Fields of one copy: field f of plane k starts at b + f fsb + k plb.
struct Copy {
  PF_GLOBAL char* b;
  int64_t fsb, plb;
  __device__ __forceinline__ PF_GLOBAL char* at(int f, int k) const {
    return b + f * fsb + (int64_t)k * plb;
  }
};

template <typename R>
__device__ __forceinline__ V4<R> load4(const Copy& c, int k, uint32_t boff) {
  V4<R> v;
#pragma unroll
  for (int a = 0; a < NP; ++a) v.v[a] = ldg<R>(c.at(a, k), boff);
  return v;
}

__device__ __forceinline__ int slot_of(int nslot, int plane) {
  return nslot == 1 ? 0 : (plane + 3) % 3;
}

// Face values of phi from LDS: the face between LDS cells (cx,cy) and its
// upper neighbour along D (slot s0 = plane k; for D = 2 the upper cell is in
// slot sp = plane k+1): face average pb and normal difference gn.
template <typename R, int D, int NSLOT>
__device__ __forceinline__ void lds_face_normal(const LdsPhi<R, NSLOT>& S, const TileGeo& G,
                                                int cx, int cy, int s0, int sp, R inv_dx,
                                                R pb[NP], R gn[NP]) {
  const int cL = G.ci(cx, cy);
  const int cU = D == 0 ? G.ci(cx + 1, cy) : (D == 1 ? G.ci(cx, cy + 1) : cL);
  const V4<R> L = S.get(s0, cL);
  const V4<R> U = D == 2 ? S.get(sp, cL) : S.get(s0, cU);
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    pb[a] = R(0.5) * (L.v[a] + U.v[a]);
    gn[a] = (U.v[a] - L.v[a]) * inv_dx;
  }
}

// Tangential face gradient components (axes in increasing order, skipping
// D), each the average of the central differences of the two face cells
// (4-point stencil); slots (sm, s0, sp) = planes (k-1, k, k+1).
template <typename R, int D, int NSLOT>
__device__ __forceinline__ void lds_face_tangential(const LdsPhi<R, NSLOT>& S, const TileGeo& G,
                                                    int cx, int cy, int sm, int s0, int sp,
                                                    R inv_4dx, R gt1[NP], R gt2[NP]) {
  const int cL = G.ci(cx, cy);
  const int cU = D == 0 ? G.ci(cx + 1, cy) : (D == 1 ? G.ci(cx, cy + 1) : cL);
  V4<R> p1L, p1U, m1L, m1U, p2L, p2U, m2L, m2U;
  if constexpr (D == 0) {  // tangential y (in plane), z (slots)
    p1L = S.get(s0, G.ci(cx, cy + 1));
    p1U = S.get(s0, G.ci(cx + 1, cy + 1));
    m1L = S.get(s0, G.ci(cx, cy - 1));
    m1U = S.get(s0, G.ci(cx + 1, cy - 1));
    p2L = S.get(sp, cL);
    p2U = S.get(sp, cU);
    m2L = S.get(sm, cL);
    m2U = S.get(sm, cU);
  } else if constexpr (D == 1) {  // tangential x, z
    p1L = S.get(s0, G.ci(cx + 1, cy));
    p1U = S.get(s0, G.ci(cx + 1, cy + 1));
    m1L = S.get(s0, G.ci(cx - 1, cy));
    m1U = S.get(s0, G.ci(cx - 1, cy + 1));
    p2L = S.get(sp, cL);
    p2U = S.get(sp, cU);
    m2L = S.get(sm, cL);
    m2U = S.get(sm, cU);
  } else {  // tangential x, y; L in plane k (s0), U in plane k+1 (sp)
    p1L = S.get(s0, G.ci(cx + 1, cy));
    p1U = S.get(sp, G.ci(cx + 1, cy));
    m1L = S.get(s0, G.ci(cx - 1, cy));
    m1U = S.get(sp, G.ci(cx - 1, cy));
    p2L = S.get(s0, G.ci(cx, cy + 1));
    p2U = S.get(sp, G.ci(cx, cy + 1));
    m2L = S.get(s0, G.ci(cx, cy - 1));
    m2U = S.get(sp, G.ci(cx, cy - 1));
  }
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    gt1[a] = ((p1L.v[a] + p1U.v[a]) - (m1L.v[a] + m1U.v[a])) * inv_4dx;
    gt2[a] = ((p2L.v[a] + p2U.v[a]) - (m2L.v[a] + m2U.v[a])) * inv_4dx;
  }
}

// Common per-item setup of both sweeps.
template <typename R>
struct ItemCtx {
  const PF_CONST DevDomain* dp;
  TileGeo G;
  Geo g;
  const PF_CONST PlaneCoef<R>* tab;
  Copy src, dst;
  uint32_t* jf;  // the item's classification word (written by the phi-sweep)
  uint32_t* jc;  // the step's counts (count_word)
  int slot;      // this item's slot of each count
  int local;     // the item's number within its domain
  DevDomain* dw;  // the descriptor, for the one word the sweeps write (pflag_ok)
};

// Item classification for the mu-sweep.  The anti-trapping current of a
// face vanishes unless a solid phase and the liquid are both present on it
// (Eq. 4 weights each solid by its product with the liquid), so it vanishes
// on every face of an item when all phi^n cells those faces touch hold no
// liquid, or all hold pure liquid.  The FP64 phi-sweep, which loads all of
// these cells (the tile, its halo ring and the planes z0-1 .. z1), records this
// per wave: byte w of the word has bit 0 set when wave w saw no liquid and
// bit 1 when it saw only liquid.  Bits are set only with the shortcuts on
// and mu not frozen; without the anti-trapping term every item qualifies.
// The phi-sweep also counts the qualifying items of the step; the split
// into two kernels is used only when those outside the chunks the phi bulk
// shortcut kept (which are light too, and are mostly the pure items the
// light kernel takes anyway) are at least kBulkMinPct percent of all items:
// a light item costs that kernel about a whole round of pure items, and
// a few of them are cheaper in the full kernel's own rounds.
constexpr uint64_t kBulkMinPct = 60;
constexpr uint32_t kBulkDone = 0x80000000u;  // item copied by the phi bulk shortcut
constexpr uint32_t kMuPure = 0x40000000u;    // item taken by the pure-item body this step
__device__ __forceinline__ bool item_jfree(uint32_t f) {
  return ((f & (f >> 8) & (f >> 16) & (f >> 24)) & 3u) != 0;
}

// Whether the FP64 mu-sweep's light body takes the item: no face of it can
// carry the anti-trapping current, and the split runs this step (uniform).
template <typename DD, typename CTX>
__device__ __forceinline__ bool item_light(const DD& d, const CTX& X) {
  if (!item_jfree(*to_const(X.jf))) return false;
  int64_t n = 0;
#pragma unroll
  for (int sl = 0; sl < kCountSlots; ++sl)
    n += (int64_t)to_const(X.jc)[count_word(kCountLight, sl)] -
         (int64_t)to_const(X.jc)[count_word(kCountFixed, sl)];
  return n * 100 >= (int64_t)d.nitems * (int64_t)kBulkMinPct;
}

// jsel < 0: every item; 0: items that need the anti-trapping current;
// 1: items that do not.  skip: items whose word has any of these bits set
// this step (taken by a kernel launched before) are passed over before
// anything else of them is read, so that a launch whose items all went
// elsewhere costs little more than one word per work group.
template <typename R>
__device__ __forceinline__ bool item_setup(DevDomain* const* doms, const int32_t* first,
                                           int ndom, int item, int t, ItemCtx<R>& X,
                                           int jsel = -1, uint32_t skip = 0) {
  const int di = find_domain(first, ndom, item);
  const PF_CONST DevDomain& d = domain_at(doms, di);
  if (!d.active) return false;  // uniform over the work group
  const int local = item - first_item(first, di);
  X.dw = to_const(doms)[di];
  X.jf = static_cast<uint32_t*>(d.jfree) + local;
  if (skip && (*to_const(X.jf) & skip)) return false;  // uniform
  X.jc = static_cast<uint32_t*>(d.jfree) + count_base(d.nitems);
  X.slot = local % kCountSlots;
  X.local = local;
  if (jsel >= 0 && item_light(d, X) != (jsel == 1)) return false;  // uniform
  X.dp = &d;
  X.G = make_tile<R>(d, local, t);
  if (!X.G.item_ok) return false;  // padding block (uniform)
  X.g = make_geo(d);
  X.tab = to_const(static_cast<const PlaneCoef<R>*>(d.coef));
  const int64_t fsb = d.fstride * (int64_t)sizeof(R), plb = d.plane * (int64_t)sizeof(R);
  X.src = Copy{to_global(static_cast<char*>(d.copy[d.cur_src])), fsb, plb};
  X.dst = Copy{to_global(static_cast<char*>(d.copy[d.cur_src ^ 1])), fsb, plb};
  return true;
}

// ------------------------------------------- bulk shortcut of the phi-sweep
//
// Each phi-sweep records, per tile and z chunk, the phase that all of the
// chunk's new cells hold purely (0..3) or 0xFF, in the flags of the copy it
// writes (pflag); the prologue withdraws a copy's flags before it is
// rewritten or after a window shift, and the sweep vouches for them again
// (pflag_ok) when it has written them; beside them, the pure phase of each
// chunk's first and last plane (pends).  A later sweep may then copy a
// chunk unchanged when it and the cells its stencils read around it
// (halo_flags: lateral chunks whole, the end planes of the chunks above and
// below; at the z ends the mirror adds nothing, a Dirichlet ghost is
// liquid) hold the same pure phase and every plane of the chunk marks that
// phase as a fixed point: every face of every cell then has zero normal
// differences, so each cell is a pure cell with A = 0, which the per-cell
// shortcut keeps exactly.
// A copied chunk's flag also carries kSame: both field copies then hold its
// phi, so when it is fixed again in the next step the copy is not needed.
constexpr uint8_t kSame = 0x10;
__device__ __forceinline__ int flag_phase(int f) { return f & 0x0F; }  // 0xFF -> 15: none

// Tile and chunk coordinates of an item (uniform over the group; made
// scalar so that the lookups below stay in scalar registers).
struct ChunkId {
  int ix, iy, iz;
};
template <typename DD>
__device__ __forceinline__ ChunkId chunk_id(const DD& d, const TileGeo& G) {
  return {__builtin_amdgcn_readfirstlane(G.x0 / G.tx), __builtin_amdgcn_readfirstlane(G.y0 / G.ty),
          __builtin_amdgcn_readfirstlane(G.z0 / d.zc)};
}
template <typename DD>
__device__ __forceinline__ int chunk_index(const DD& d, const ChunkId& c) {
  return (c.iz * d.nty + c.iy) * d.ntx + c.ix;  // < 2^31: the layout bounds the items
}

template <typename DD>
__device__ __forceinline__ void dd_mark_flags(const DD& d, DevDomain* dw) {
  // the flags of the copy being written are complete once the sweep ends
  // (the descriptor is read through the constant address space; this one
  // word, which the sweeps never read, is written through its plain pointer)
  to_global(&dw->pflag_ok[d.cur_src ^ 1])[0] = 1;
}

// The flags that decide whether the cells a chunk's stencils read around
// it hold one pure phase: of the chunk and its 8 lateral neighbours the
// whole-chunk flag, of the 9 chunks below and the 9 above the end-plane flag
// (only their top / bottom plane lies within one cell of the chunk).
// Periodic in x and y; a z neighbour outside the domain reads the chunk
// itself (the mirror repeats its own end plane).  All 27 bytes are loaded
// before any is tested, so that the loads overlap instead of taking one
// round trip each.
template <typename DD>
__device__ __forceinline__ void halo_flags(const DD& d, const PF_CONST uint8_t* f,
                                           const PF_CONST uint8_t* e, const ChunkId& c, int v[27]) {
  int jx[3], jy[3], jz[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int x = c.ix + i - 1, y = c.iy + i - 1, z = c.iz + i - 1;
    jx[i] = x < 0 ? d.ntx - 1 : (x == d.ntx ? 0 : x);
    jy[i] = y < 0 ? d.nty - 1 : (y == d.nty ? 0 : y);
    jz[i] = z < 0 || z >= d.nzc ? c.iz : z;
  }
#pragma unroll
  for (int i = 0; i < 27; ++i)
    v[i] = (i / 9 == 1 ? f : e)[(jz[i / 9] * d.nty + jy[(i / 3) % 3]) * d.ntx + jx[i % 3]];
}
// Whether halo_flags v all say phase a (below: top plane; lateral: whole
// chunk; above: bottom plane).
__device__ __forceinline__ bool halo_is(const int v[27], int a) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int p = i < 9 ? v[i] >> 4 : (i < 18 ? flag_phase(v[i]) : v[i] & 0x0F);
    ok = ok && p == a;
  }
  return ok;
}

// The phase of a bulk chunk that may be copied, or -1 (uniform over the
// group): the chunk holds phase a purely, so do the cells its stencils
// read around it (halo_flags; the ghost plane of a Dirichlet top is
// liquid), and every plane of the chunk marks a as a fixed point.
template <typename DD, typename TAB>
__device__ __forceinline__ int bulk_fixed_phase(const DD& d, const ChunkId& c, int z0,
                                                const TAB* tab) {
  if (!d.pflag_ok[d.cur_src]) return -1;
  const PF_CONST uint8_t* f = to_const(static_cast<const uint8_t*>(d.pflag[d.cur_src]));
  const PF_CONST uint8_t* e = to_const(static_cast<const uint8_t*>(d.pends[d.cur_src]));
  const int a = flag_phase(f[chunk_index(d, c)]);
  if (a >= NP) return -1;
  if (c.iz + 1 >= d.nzc && d.top_bc && a != LQ) return -1;
  int v[27];
  halo_flags(d, f, e, c, v);
  const bool ok = ((tab[z0].chunk_fixed >> a) & 1) != 0 && halo_is(v, a);
  return ok ? a : -1;
}

// The phase a when the item's chunk and the cells its stencils read around
// it hold phase a purely both before and after this step's phi-sweep (the
// flags of the source copy, valid unless withdrawn, and those the sweep has
// just written for the copy it wrote), else -1.  Then phi^n = phi^{n+1} =
// e_a on every cell the mu-sweep reads for the item (at the z ends the
// mirror adds nothing, the ghost plane of a Dirichlet top is liquid).
// Uniform over the group.
template <typename DD>
__device__ __forceinline__ int mu_pure_phase(const DD& d, const ChunkId& c) {
  if (!d.pflag_ok[d.cur_src]) return -1;
  const int s0 = d.cur_src, s1 = d.cur_src ^ 1;
  const PF_CONST uint8_t* f1 = to_const(static_cast<const uint8_t*>(d.pflag[s1]));
  const int idx = chunk_index(d, c);
  const int a = flag_phase(f1[idx]);
  if (a >= NP) return -1;
  if (c.iz + 1 >= d.nzc && d.top_bc && a != LQ) return -1;
  int v[27];
  // after the sweep first: most items fail there
  halo_flags(d, f1, to_const(static_cast<const uint8_t*>(d.pends[s1])), c, v);
  if (!halo_is(v, a)) return -1;
  halo_flags(d, to_const(static_cast<const uint8_t*>(d.pflag[s0])),
             to_const(static_cast<const uint8_t*>(d.pends[s0])), c, v);
  return halo_is(v, a) ? a : -1;
}

// The phase a cell holds purely (phi = e_a exactly), or -1.
template <typename R>
__device__ __forceinline__ int pure_phase(const R o[NP]) {
  int a = -1, ones = 0, zeros = 0;
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    ones += o[b] == R(1);
    zeros += o[b] == R(0);
    if (o[b] == R(1)) a = b;
  }
  return ones == 1 && zeros == NP - 1 ? a : -1;
}

// Combination over a wave of the lanes' pure phases (-2: lane wrote no
// cell): -2 if no lane wrote, the common phase, or -1.
__device__ __forceinline__ int wave_pure_phase(int po) {
  if (!__any(po != -2)) return -2;
  for (int a = 0; a < NP; ++a)
    if (__all(po == a || po == -2)) return a;
  return -1;
}

// ============================================================ phi-sweep

template <typename R, bool ANISO>
__device__ __forceinline__ void phi_tiled_body(DevDomain* const* doms, const int32_t* first,
                                               int ndom, int total, const uint32_t* words) {
  constexpr int NSLOT = ANISO ? 3 : 1;
  constexpr int AHEAD = ANISO ? 2 : 1;  // plane loaded during iteration k: k + AHEAD
  __shared__ LdsPhi<R, NSLOT> s_phi;
  __shared__ R s_qx[NP][kMaxFx];  // Q of the x faces (their share in the cell above)
  __shared__ R s_qy[NP][kFyCap<R>];
  __shared__ uint8_t s_jw[4];          // per-wave bytes of the item's classification word
  __shared__ int8_t s_pw[4];           // per-wave pure phase of the outputs (pure_phase_flag)
  __shared__ int8_t s_pe[2][4];        // the same for the first and last plane
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    // a single domain's launch passes its item words: a chunk the bulk
    // kernel kept is passed over after one load
    if (words && (to_const(words)[item] & kBulkDone)) continue;
    ItemCtx<R> X;
    // in a pack (no item words), the chunks copied unchanged by
    // phi_bulk_kernel: FP64 passes them over before the tile is set up,
    // FP32 after it (the early test cost the FP32 anisotropic sweep 0.4%)
    if (!item_setup(doms, first, ndom, item, t, X, -1, sizeof(R) == 8 ? kBulkDone : 0u)) continue;
    const TileGeo& G = X.G;
    const Geo& g = X.g;
    const auto& P = kparams<R>(*X.dp);
    const Copy& src = X.src;
    const Copy& dst = X.dst;
    const R inv_dx = (R)P.inv_dx, inv_4dx = (R)P.inv_4dx;
    const bool shortcut = P.shortcuts != 0;
    const int kstart = G.z0 - 1;
    const PF_CONST DevDomain& dd = *X.dp;
    const ChunkId cid = chunk_id(dd, G);

    if (*to_const(X.jf) & kBulkDone) continue;
    // pure phase of this thread's outputs so far (-2: none, -1: mixed), and
    // of its outputs on the first and last plane: bytes 0, 1, 2 hold each + 2
    int pst = 0;

    // liquid content of every phi^n cell this item loads (item_jfree; the
    // FP64 mu-sweep only)
    constexpr bool CLASSIFY = sizeof(R) == 8;
    bool no_liq = true, only_liq = true;
    const auto note = [&](const V4<R>& v) {
      if constexpr (CLASSIFY) {
        no_liq = no_liq && v.v[LQ] == R(0);
        only_liq = only_liq && v.v[0] == R(0) && v.v[1] == R(0) && v.v[2] == R(0);
      }
    };

    // prime the LDS ring with planes kstart-1 .. kstart+1 (ANISO) or kstart
    for (int p = kstart - (NSLOT == 3 ? 1 : 0); p <= kstart + (NSLOT == 3 ? 1 : 0); ++p) {
      const int pc = g.zc(p), sl = slot_of(NSLOT, p);
      const V4<R> vo = load4<R>(src, pc, G.own_b);
      note(vo);
      s_phi.put(sl, G.own_c, vo);
      if (G.halo_c >= 0) {
        const V4<R> vh = load4<R>(src, pc, G.halo_b);
        note(vh);
        s_phi.put(sl, G.halo_c, vh);
      }
    }
    V4<R> own_k = load4<R>(src, g.zc(kstart), G.own_b);
    __syncthreads();

    R Qzl[NP];  // share of the z face below the current plane
#pragma unroll
    for (int a = 0; a < NP; ++a) Qzl[a] = R(0);

    for (int k = kstart; k < G.z1; ++k) {
      const bool cells = k >= G.z0;  // kstart only evaluates the z face above it
      const int sm = slot_of(NSLOT, k - 1), s0 = slot_of(NSLOT, k), sp = slot_of(NSLOT, k + 1);
      // issue the loads of plane k+AHEAD (own column and halo cell)
      const int pa = g.zc(k + AHEAD);
      const V4<R> nxt_own = load4<R>(src, pa, G.own_b);
      V4<R> nxt_halo;
      if (G.halo_c >= 0) nxt_halo = load4<R>(src, pa, G.halo_b);
      R mc[NM] = {R(0), R(0)};
      R Px[NP] = {}, Py[NP] = {};  // shares of the own upper x and y faces
      if (cells) {
        mc[0] = ldg<R>(src.at(4, k), G.own_b);
        mc[1] = ldg<R>(src.at(5, k), G.own_b);
        // x faces: own upper face, plus the tile's lower edge faces, taken
        // by the first ty lanes of wave (k+1) mod 4 (same code path for
        // both); y faces likewise with the first tx lanes of wave k mod 4.
        // Rotating the edge duty over the planes keeps any one wave from
        // carrying the extra faces of every plane.
        const bool ex = wave == ((k + 1) & 3) && lane < G.ty && G.y0 + lane < g.ny;
        const bool ey = wave == (k & 3) && lane < G.tx && G.x0 + lane < g.nx;
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          const bool edge = r == 1;
          if (edge ? !ex : !G.valid) continue;
          const int cx = edge ? 0 : G.lx + 1, cy = edge ? lane + 1 : G.ly + 1;
          const int fo = edge ? lane * (G.tx + 1) : G.ly * (G.tx + 1) + G.lx + 1;
          R pb[NP], gn[NP], gt1[NP] = {}, gt2[NP] = {}, F[NP] = {}, S[NP] = {};
          lds_face_normal<R, 0>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
          if (!(shortcut && zero_normal(gn))) {
            if constexpr (ANISO) lds_face_tangential<R, 0>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
            phi_face<R, ANISO, 0>(P, pb, gn, gt1, gt2, F, S);
          }
          R Pv[NP], Qv[NP];
          face_pq<R>(F, S, inv_dx, Pv, Qv);
#pragma unroll
          for (int a = 0; a < NP; ++a) {
            s_qx[a][fo] = Qv[a];
            if (!edge) Px[a] = Pv[a];
          }
        }
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          const bool edge = r == 1;
          if (edge ? !ey : !G.valid) continue;
          const int cx = edge ? lane + 1 : G.lx + 1, cy = edge ? 0 : G.ly + 1;
          const int fo = edge ? lane : (G.ly + 1) * G.tx + G.lx;
          R pb[NP], gn[NP], gt1[NP] = {}, gt2[NP] = {}, F[NP] = {}, S[NP] = {};
          lds_face_normal<R, 1>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
          if (!(shortcut && zero_normal(gn))) {
            if constexpr (ANISO) lds_face_tangential<R, 1>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
            phi_face<R, ANISO, 1>(P, pb, gn, gt1, gt2, F, S);
          }
          R Pv[NP], Qv[NP];
          face_pq<R>(F, S, inv_dx, Pv, Qv);
#pragma unroll
          for (int a = 0; a < NP; ++a) {
            s_qy[a][fo] = Qv[a];
            if (!edge) Py[a] = Pv[a];
          }
        }
      }
      // z face above plane k (zero on the z boundaries)
      R Pz[NP] = {}, Qzu[NP] = {};
      if (g.zface(k)) {
        R Fzu[NP] = {}, Szu[NP] = {};
        R pb[NP], gn[NP], gt1[NP] = {}, gt2[NP] = {};
        if constexpr (ANISO) {
          lds_face_normal<R, 2>(s_phi, G, G.lx + 1, G.ly + 1, s0, sp, inv_dx, pb, gn);
        } else {
          // own column at k (registers) and k+1 (just loaded)
#pragma unroll
          for (int a = 0; a < NP; ++a) {
            pb[a] = R(0.5) * (own_k.v[a] + nxt_own.v[a]);
            gn[a] = (nxt_own.v[a] - own_k.v[a]) * inv_dx;
          }
        }
        if (!(shortcut && zero_normal(gn))) {
          if constexpr (ANISO)
            lds_face_tangential<R, 2>(s_phi, G, G.lx + 1, G.ly + 1, sm, s0, sp, inv_4dx, gt1, gt2);
          phi_face<R, ANISO, 2>(P, pb, gn, gt1, gt2, Fzu, Szu);
        }
        face_pq<R>(Fzu, Szu, inv_dx, Pz, Qzu);
      }
      V4<R> ownv;
      if constexpr (ANISO) ownv = s_phi.get(s0, G.own_c);
      else ownv = own_k;
      __syncthreads();  // B1: faces visible; LDS plane slots of k-1 (or k) free
      {
        const int sl = slot_of(NSLOT, k + AHEAD);
        s_phi.put(sl, G.own_c, nxt_own);
        note(nxt_own);
        if (G.halo_c >= 0) {
          s_phi.put(sl, G.halo_c, nxt_halo);
          note(nxt_halo);
        }
      }
      if (cells && G.valid) {
        const int fl = G.ly * (G.tx + 1) + G.lx;  // lower x face
        const int yl = G.ly * G.tx + G.lx;        // lower y face
        R A[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a)
          A[a] = ((Px[a] + s_qx[a][fl]) + (Py[a] + s_qy[a][yl])) + (Pz[a] + Qzl[a]);
        double out[NP];
        if (shortcut && pure_cell_fixed(ownv.v, A, X.tab[k].pure_fixed)) {
#pragma unroll
          for (int a = 0; a < NP; ++a) out[a] = (double)ownv.v[a];
        } else {
          phi_cell<R>(P, X.tab[k], ownv.v, mc, A, out);
        }
        R o[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          o[a] = (R)out[a];
          stg<R>(dst.at(a, k), G.own_b, o[a]);
        }
        const int pa = pure_phase(o);
        const int po = (pst & 0xFF) - 2;
        pst = (pst & ~0xFF) | ((po == -2 ? pa : (po == pa ? po : -1)) + 2);
        if (k == G.z0) pst = (pst & ~0xFF00) | (pa + 2) << 8;
        if (k == G.z1 - 1) pst = (pst & ~0xFF0000) | (pa + 2) << 16;
      }
#pragma unroll
      for (int a = 0; a < NP; ++a) Qzl[a] = Qzu[a];
      if constexpr (!ANISO) own_k = nxt_own;
      __syncthreads();  // B2: LDS plane and faces consumed
    }
    // end of the item: the pure phase of its outputs (for the next step's
    // bulk shortcut) and, in FP64, the mu-sweep's classification
    {
      const int wp = wave_pure_phase((pst & 0xFF) - 2);
      const int we0 = wave_pure_phase((pst >> 8 & 0xFF) - 2), we1 = wave_pure_phase((pst >> 16) - 2);
      uint32_t b = 0;
      if constexpr (CLASSIFY)
        if (shortcut && !P.mu_frozen)
          b = !P.antitrap ? 3u : (__all(no_liq) ? 1u : 0u) | (__all(only_liq) ? 2u : 0u);
      if (lane == 0) {
        s_pw[wave] = (int8_t)wp;
        s_pe[0][wave] = (int8_t)we0;
        s_pe[1][wave] = (int8_t)we1;
        s_jw[wave] = (uint8_t)b;
      }
      __syncthreads();
      if (t == 0) {
        const auto group = [](const int8_t* p) {
          int ph = -2;
          for (int w = 0; w < 4; ++w) {
            const int v = p[w];
            ph = v == -2 ? ph : (ph == -2 || ph == v ? v : -1);
          }
          return ph;
        };
        const int ph = group(s_pw), e0 = group(s_pe[0]), e1 = group(s_pe[1]);
        const int idx = chunk_index(dd, cid);
        static_cast<uint8_t*>(dd.pflag[dd.cur_src ^ 1])[idx] = ph >= 0 ? (uint8_t)ph : (uint8_t)0xFF;
        static_cast<uint8_t*>(dd.pends[dd.cur_src ^ 1])[idx] =
            (uint8_t)((e1 >= 0 ? e1 : 0xF) << 4 | (e0 >= 0 ? e0 : 0xF));
        dd_mark_flags(dd, X.dw);
        if constexpr (CLASSIFY) {
          const uint32_t w = (uint32_t)s_jw[0] | (uint32_t)s_jw[1] << 8 | (uint32_t)s_jw[2] << 16 |
                             (uint32_t)s_jw[3] << 24;
          *to_global(X.jf) = w;
          if (item_jfree(w)) atomicAdd(X.jc + count_word(kCountLight, X.slot), 1u);
        }
      }
    }
  }
}

// One kernel per precision and stencil.  The FP32 anisotropic sweep, which
// is bound by its arithmetic, is held to 96 VGPRs so that five waves fit per
// SIMD (it needs 98 otherwise, which allows four).
__global__ __launch_bounds__(kTileThreads) void phi_tiled_f64(DevDomain* const* doms,
                                                              const int32_t* first, int ndom,
                                                              int total, const uint32_t* words) {
  phi_tiled_body<double, false>(doms, first, ndom, total, words);
}
__global__ __launch_bounds__(kTileThreads) void phi_tiled_f64_aniso(DevDomain* const* doms,
                                                                    const int32_t* first, int ndom,
                                                                    int total, const uint32_t* words) {
  phi_tiled_body<double, true>(doms, first, ndom, total, words);
}
__global__ __launch_bounds__(kTileThreads) void phi_tiled_f32(DevDomain* const* doms,
                                                              const int32_t* first, int ndom,
                                                              int total, const uint32_t* words) {
  phi_tiled_body<float, false>(doms, first, ndom, total, words);
}
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(5))) void
phi_tiled_f32_aniso(DevDomain* const* doms, const int32_t* first, int ndom, int total, const uint32_t* words) {
  phi_tiled_body<float, true>(doms, first, ndom, total, words);
}

// Bulk shortcut of the phi-sweep, launched before it over the same items:
// a chunk that bulk_fixed_phase finds fixed is copied unchanged, its flags
// and (FP64) the mu-sweep's classification are written, and its word is
// marked kBulkDone so that the sweep passes it over; every other item's
// word is cleared for the sweep to fill.
// phi_bulk_kernel takes `per` consecutive items per wave, and the work
// group adds the counts of its items to the step's counters once: an
// increment of one word is serialised (about 12 ns each), and one per item
// made the kernel wait on the counters (55 us for the 32768 items of a
// 512x512x1024 FP32 domain).  More items per wave cut the increments
// further but run the waves' tests one after another, so a launch takes
// one item per wave until its waves would fill the chip more than once
// (bulk_items_per_wave).
constexpr int kBulkMaxPerWave = 4, kBulkFillWaves = 8192;
inline int bulk_items_per_wave(int total) {
  const int per = total / kBulkFillWaves;
  return per < 1 ? 1 : (per > kBulkMaxPerWave ? kBulkMaxPerWave : per);
}

template <typename R>
__global__ __launch_bounds__(kTileThreads) void phi_bulk_kernel(DevDomain* const* doms,
                                                                const int32_t* first, int ndom,
                                                                int total, int per) {
  // the test is a few dependent loads, so each wave takes its own items
  // (four waves' tests in flight per work group)
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // scalar
  const int lane = threadIdx.x & 63;
  // counts of this wave's items not yet added: fixed, copied, light, and
  // the domain's counter words they belong to (uniform over the wave)
  __shared__ uint32_t* s_jc[kTileWaves];
  __shared__ uint32_t s_n[kTileWaves][3];
  uint32_t* jc = nullptr;
  int slot = 0;
  uint32_t n[3] = {0u, 0u, 0u};
  const auto flush = [&]() {
    if (lane == 0 && jc) {
      if (n[0]) atomicAdd(jc + count_word(kCountFixed, slot), n[0]);
      if (n[1]) atomicAdd(jc + count_word(kCountCopied, slot), n[1]);
      if (n[2]) atomicAdd(jc + count_word(kCountLight, slot), n[2]);
    }
    n[0] = n[1] = n[2] = 0u;
  };
  const int base = (blockIdx.x * kTileWaves + wave) * per;
  for (int item = base; item < base + per && item < total; ++item) {
    ItemCtx<R> X;
    if (!item_setup(doms, first, ndom, item, lane, X)) continue;  // uniform over the wave
    if (X.jc != jc) {  // another domain (a pack): add what the last one counted
      flush();
      jc = X.jc;
      slot = X.slot;
    }
    const auto& P = kparams<R>(*X.dp);
    const PF_CONST DevDomain& dd = *X.dp;
    const ChunkId cid = chunk_id(dd, X.G);
    const int z0 = __builtin_amdgcn_readfirstlane(X.G.z0);
    const int fixed = P.shortcuts ? bulk_fixed_phase(dd, cid, z0, X.tab) : -1;
    if (fixed < 0) {
      if (lane == 0) *to_global(X.jf) = 0u;
      continue;
    }
    // unless both copies already hold the chunk (copied or kept in the
    // previous step too), copy it into the one this step writes; the wave
    // takes the tile's columns kTileWaves at a time
    const bool same =
        to_const(static_cast<const uint8_t*>(dd.pflag[dd.cur_src]))[chunk_index(dd, cid)] & kSame;
    if (!same) {
      ++n[1];
#pragma unroll 1
      for (int c = lane; c < kTileThreads; c += 64) {
        const TileGeo Gc = make_tile<R>(dd, X.local, c);
        if (!Gc.valid) continue;
#pragma unroll 4
        for (int k = Gc.z0; k < Gc.z1; ++k) {
          const V4<R> v = load4<R>(X.src, k, Gc.own_b);
#pragma unroll
          for (int a = 0; a < NP; ++a) stg<R>(X.dst.at(a, k), Gc.own_b, v.v[a]);
        }
      }
    }
    ++n[0];
    uint32_t w = 0;
    if constexpr (sizeof(R) == 8) {  // the mu-sweep's classification (item_jfree)
      const uint32_t b = P.mu_frozen ? 0u : (!P.antitrap ? 3u : (fixed == LQ ? 2u : 1u));
      w = b * 0x01010101u;
      if (item_jfree(w)) ++n[2];
    }
    if (lane == 0) {
      static_cast<uint8_t*>(dd.pflag[dd.cur_src ^ 1])[chunk_index(dd, cid)] =
          (uint8_t)(fixed | kSame);
      static_cast<uint8_t*>(dd.pends[dd.cur_src ^ 1])[chunk_index(dd, cid)] = (uint8_t)(fixed << 4 | fixed);
      dd_mark_flags(dd, X.dw);
      *to_global(X.jf) = w | kBulkDone;
    }
  }
  // the waves of a work group that counted for one domain add their counts
  // together, the others each their own
  if (lane == 0) {
    s_jc[wave] = jc;
    s_n[wave][0] = n[0];
    s_n[wave][1] = n[1];
    s_n[wave][2] = n[2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 0; v < kTileWaves; ++v) {
      uint32_t* j = s_jc[v];
      if (!j) continue;
      uint32_t t[3] = {s_n[v][0], s_n[v][1], s_n[v][2]};
      for (int u = v + 1; u < kTileWaves; ++u)
        if (s_jc[u] == j) {
          for (int q = 0; q < 3; ++q) t[q] += s_n[u][q];
          s_jc[u] = nullptr;
        }
      const int sl = (int)(blockIdx.x % kCountSlots);
      if (t[0]) atomicAdd(j + count_word(kCountFixed, sl), t[0]);
      if (t[1]) atomicAdd(j + count_word(kCountCopied, sl), t[1]);
      if (t[2]) atomicAdd(j + count_word(kCountLight, sl), t[2]);
    }
  }
}

// ============================================================= mu-sweep

// phi^{n+1} - phi^n of the solid phases summed over the two cells of a
// face, for dphi/dt (both planes from LDS).
template <typename R>
__device__ __forceinline__ void face_dphi(const V4<R>& L1, const V4<R>& U1, const V4<R>& L0,
                                          const V4<R>& U0, R dph[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) dph[a] = (L1.v[a] - L0.v[a]) + (U1.v[a] - U0.v[a]);
}

template <typename R>
__device__ __forceinline__ void mu_tiled_body(DevDomain* const* doms, const int32_t* first, int ndom,
                                              int total, const uint32_t* words) {
  constexpr int NSLOT = 3, AHEAD = 2;
  __shared__ LdsPhi<R, NSLOT> s_phi;
  __shared__ LdsMu<R> s_mu;         // mu^n of plane k
  __shared__ LdsPhi<R, 1> s_p1;     // phi^{n+1} of plane k
  __shared__ R s_fx[NM][kMaxFx];
  __shared__ R s_fy[NM][kFyCap<R>];
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    // a single domain's launch passes its item words: an FP64 item the
    // pure-item launch took is passed over after one load (in FP32 the extra
    // load ahead of every item's set-up cost more than it saved: c3 +0.8%)
    if (sizeof(R) == 8 && words && (to_const(words)[item] & kMuPure)) continue;
    ItemCtx<R> X;
    // FP64: the items that need the anti-trapping current (mu_light_f64
    // takes the rest); FP32: every item
    if (!item_setup(doms, first, ndom, item, t, X, sizeof(R) == 8 ? 0 : -1)) continue;
    const TileGeo& G = X.G;
    const Geo& g = X.g;
    const auto& P = kparams<R>(*X.dp);
    const Copy& src = X.src;  // phi^n (fields 0-3), mu^n (4-5)
    const Copy& dst = X.dst;  // phi^{n+1} (written by the phi-sweep), mu^{n+1}
    const R inv_dx = (R)P.inv_dx, inv_4dx = (R)P.inv_4dx;
    const bool antitrap = P.antitrap != 0;
    // FP64: the three own faces side by side (more independent work per
    // wave at two waves per SIMD); FP32, held to 128 VGPRs, one at a time
    constexpr bool ILP = sizeof(R) == 8;
    const int kstart = G.z0 - 1;

    if (P.mu_frozen) {  // mu^{n+1} = mu^n (tests of the phi part only)
      if (G.valid)
        for (int k = G.z0; k < G.z1; ++k) {
          stg<R>(dst.at(4, k), G.own_b, ldg<R>(src.at(4, k), G.own_b));
          stg<R>(dst.at(5, k), G.own_b, ldg<R>(src.at(5, k), G.own_b));
        }
      continue;
    }
    // items pure in one phase: taken by mu_light_f64 / mu_pure_f32 (launched first)
    if (P.shortcuts && (*to_const(X.jf) & kMuPure)) continue;

    // lane l of the edge wave takes the lower-edge face of tile row l (x)
    // or tile column l (y), between x0-1 and x0 / y0-1 and y0
    const bool ex_ok = lane < G.ty && G.y0 + lane < g.ny;
    const bool ey_ok = lane < G.tx && G.x0 + lane < g.nx;

    for (int p = kstart - 1; p <= kstart + 1; ++p) {
      const int pc = g.zc(p), sl = slot_of(NSLOT, p);
      s_phi.put(sl, G.own_c, load4<R>(src, pc, G.own_b));
      if (G.halo_c >= 0) s_phi.put(sl, G.halo_c, load4<R>(src, pc, G.halo_b));
    }
    // mu^n of plane kstart into LDS (own column also kept in registers),
    // phi^{n+1} of the own column at plane kstart
    const int kc0 = g.zc(kstart);
    R ownm[NM] = {ldg<R>(src.at(4, kc0), G.own_b), ldg<R>(src.at(5, kc0), G.own_b)};
    s_mu.put(G.own_c, ownm);
    if (G.halo_c >= 0) {
      const R hm[NM] = {ldg<R>(src.at(4, kc0), G.halo_b), ldg<R>(src.at(5, kc0), G.halo_b)};
      s_mu.put(G.halo_c, hm);
    }
    V4<R> own1 = load4<R>(dst, kc0, G.own_b);
    s_p1.put(0, G.own_c, own1);
    if (G.halo_c >= 0) s_p1.put(0, G.halo_c, load4<R>(dst, kc0, G.halo_b));
    __syncthreads();

    R Pzl[NM] = {R(0), R(0)};
    for (int k = kstart; k < G.z1; ++k) {
      const bool cells = k >= G.z0;
      const int sm = slot_of(NSLOT, k - 1), s0 = slot_of(NSLOT, k), sp = slot_of(NSLOT, k + 1);
      const int pa = g.zc(k + AHEAD);
      const V4<R> nxt_own = load4<R>(src, pa, G.own_b);
      V4<R> nxt_halo;
      if (G.halo_c >= 0) nxt_halo = load4<R>(src, pa, G.halo_b);
      // plane k+1: mu^n (own column and halo cell; the own value also feeds
      // the z face above k) and phi^{n+1} of the own column
      const int k1 = g.zp(k);
      const R upm[NM] = {ldg<R>(src.at(4, k1), G.own_b), ldg<R>(src.at(5, k1), G.own_b)};
      R nxt_hm[NM] = {R(0), R(0)};
      if (G.halo_c >= 0) {
        nxt_hm[0] = ldg<R>(src.at(4, k1), G.halo_b);
        nxt_hm[1] = ldg<R>(src.at(5, k1), G.halo_b);
      }
      const V4<R> up1 = load4<R>(dst, k1, G.own_b);
      V4<R> nxt_p1h;
      if (G.halo_c >= 0) nxt_p1h = load4<R>(dst, k1, G.halo_b);
      const int kk = k < 0 ? 0 : k;
      const auto& C = X.tab[kk];
      // x face between LDS cells (cx,cy), (cx+1,cy) and y face between
      // (cx,cy), (cx,cy+1) of plane k, with their anti-trapping terms
      const auto j_x = [&](int cx, int cy, const R pb[NP], const R gn[NP], const R mL[NM],
                           const R mU[NM], R Phi[NM]) {
        R gt1[NP], gt2[NP], dph[3];
        face_dphi<R>(s_p1.get(0, G.ci(cx, cy)), s_p1.get(0, G.ci(cx + 1, cy)),
                     s_phi.get(s0, G.ci(cx, cy)), s_phi.get(s0, G.ci(cx + 1, cy)), dph);
        {
          lds_face_tangential<R, 0>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
          mu_face_j<R, false>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
        }
      };
      const auto j_y = [&](int cx, int cy, const R pb[NP], const R gn[NP], const R mL[NM],
                           const R mU[NM], R Phi[NM]) {
        R gt1[NP], gt2[NP], dph[3];
        face_dphi<R>(s_p1.get(0, G.ci(cx, cy)), s_p1.get(0, G.ci(cx, cy + 1)),
                     s_phi.get(s0, G.ci(cx, cy)), s_phi.get(s0, G.ci(cx, cy + 1)), dph);
        {
          lds_face_tangential<R, 1>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
          mu_face_j<R, false>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
        }
      };
      R Pzu[NM] = {R(0), R(0)};  // z face above plane k
      if constexpr (ILP) {
        // The three faces above the own cell (x, y, and z above plane k) are
        // independent: their diffusive parts are evaluated side by side; the
        // anti-trapping terms follow where needed, re-reading the face values
        // so that no face's inputs stay live across the others.
        const bool own = cells && G.valid;
        const bool zf = g.zface(k);
        const int ox = G.lx + 1, oy = G.ly + 1;
        R Phx[NM], Phy[NM];
        bool jx = false, jy = false, jz = false;
        if (own) {
          R pbx[NP], gnx[NP], pby[NP], gny[NP], mUx[NM], mUy[NM];
          lds_face_normal<R, 0>(s_phi, G, ox, oy, s0, sp, inv_dx, pbx, gnx);
          lds_face_normal<R, 1>(s_phi, G, ox, oy, s0, sp, inv_dx, pby, gny);
          s_mu.get(G.ci(ox + 1, oy), mUx);
          s_mu.get(G.ci(ox, oy + 1), mUy);
          mu_face_diff<R, false>(P, C, pbx, ownm, mUx, Phx);
          mu_face_diff<R, false>(P, C, pby, ownm, mUy, Phy);
          jx = antitrap && mu_face_needs_j(pbx);
          jy = antitrap && mu_face_needs_j(pby);
        }
        if (zf) {
          R pbz[NP], gnz[NP];
          lds_face_normal<R, 2>(s_phi, G, ox, oy, s0, sp, inv_dx, pbz, gnz);
          mu_face_diff<R, true>(P, C, pbz, ownm, upm, Pzu);
          jz = antitrap && mu_face_needs_j(pbz);
        }
        if (jx) {
          R pb[NP], gn[NP], mU[NM];
          lds_face_normal<R, 0>(s_phi, G, ox, oy, s0, sp, inv_dx, pb, gn);
          s_mu.get(G.ci(ox + 1, oy), mU);
          j_x(ox, oy, pb, gn, ownm, mU, Phx);
        }
        if (jy) {
          R pb[NP], gn[NP], mU[NM];
          lds_face_normal<R, 1>(s_phi, G, ox, oy, s0, sp, inv_dx, pb, gn);
          s_mu.get(G.ci(ox, oy + 1), mU);
          j_y(ox, oy, pb, gn, ownm, mU, Phy);
        }
        if (jz) {
          R pb[NP], gn[NP], gt1[NP], gt2[NP], dph[3];
          lds_face_normal<R, 2>(s_phi, G, ox, oy, s0, sp, inv_dx, pb, gn);
          const V4<R> L0 = s_phi.get(s0, G.own_c), U0 = s_phi.get(sp, G.own_c);
  #pragma unroll
          for (int a = 0; a < 3; ++a) dph[a] = (own1.v[a] - L0.v[a]) + (up1.v[a] - U0.v[a]);
          {
            lds_face_tangential<R, 2>(s_phi, G, ox, oy, sm, s0, sp, inv_4dx, gt1, gt2);
            mu_face_j<R, true>(P, C, pb, gn, gt1, gt2, dph, ownm, upm, Pzu);
          }
        }
        if (own) {
          const int fx = G.ly * (G.tx + 1) + G.lx + 1, fy = (G.ly + 1) * G.tx + G.lx;
          s_fx[0][fx] = Phx[0];
          s_fx[1][fx] = Phx[1];
          s_fy[0][fy] = Phy[0];
          s_fy[1][fy] = Phy[1];
        }
        // the tile's lower-edge faces: lane l of one wave per direction,
        // rotating with the plane (x edge: wave (k+1) mod 4, y edge: k mod 4)
        if (cells && ex_ok && wave == ((k + 1) & 3)) {
          const int cx = 0, cy = lane + 1;
          R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
          lds_face_normal<R, 0>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
          s_mu.get(G.ci(cx, cy), mL);
          s_mu.get(G.ci(cx + 1, cy), mU);
          mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
          if (antitrap && mu_face_needs_j(pb)) j_x(cx, cy, pb, gn, mL, mU, Phi);
          s_fx[0][lane * (G.tx + 1)] = Phi[0];
          s_fx[1][lane * (G.tx + 1)] = Phi[1];
        }
        if (cells && ey_ok && wave == (k & 3)) {
          const int cx = lane + 1, cy = 0;
          R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
          lds_face_normal<R, 1>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
          s_mu.get(G.ci(cx, cy), mL);
          s_mu.get(G.ci(cx, cy + 1), mU);
          mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
          if (antitrap && mu_face_needs_j(pb)) j_y(cx, cy, pb, gn, mL, mU, Phi);
          s_fy[0][lane] = Phi[0];
          s_fy[1][lane] = Phi[1];
        }
      } else {
        if (cells) {
          const bool ex = ex_ok && wave == ((k + 1) & 3);
          const bool ey = ey_ok && wave == (k & 3);
  #pragma unroll 1
          for (int r = 0; r < 2; ++r) {
            const bool edge = r == 1;
            if (edge ? !ex : !G.valid) continue;
            const int cx = edge ? 0 : G.lx + 1, cy = edge ? lane + 1 : G.ly + 1;
            const int fo = edge ? lane * (G.tx + 1) : G.ly * (G.tx + 1) + G.lx + 1;
            R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
            lds_face_normal<R, 0>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
            s_mu.get(G.ci(cx, cy), mL);
            s_mu.get(G.ci(cx + 1, cy), mU);
            mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
            if (antitrap && mu_face_needs_j(pb)) {
              R gt1[NP], gt2[NP], dph[3];
              face_dphi<R>(s_p1.get(0, G.ci(cx, cy)), s_p1.get(0, G.ci(cx + 1, cy)),
                           s_phi.get(s0, G.ci(cx, cy)), s_phi.get(s0, G.ci(cx + 1, cy)), dph);
              {
                lds_face_tangential<R, 0>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
                mu_face_j<R, false>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
              }
            }
            s_fx[0][fo] = Phi[0];
            s_fx[1][fo] = Phi[1];
          }
  #pragma unroll 1
          for (int r = 0; r < 2; ++r) {
            const bool edge = r == 1;
            if (edge ? !ey : !G.valid) continue;
            const int cx = edge ? lane + 1 : G.lx + 1, cy = edge ? 0 : G.ly + 1;
            const int fo = edge ? lane : (G.ly + 1) * G.tx + G.lx;
            R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
            lds_face_normal<R, 1>(s_phi, G, cx, cy, s0, sp, inv_dx, pb, gn);
            s_mu.get(G.ci(cx, cy), mL);
            s_mu.get(G.ci(cx, cy + 1), mU);
            mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
            if (antitrap && mu_face_needs_j(pb)) {
              R gt1[NP], gt2[NP], dph[3];
              face_dphi<R>(s_p1.get(0, G.ci(cx, cy)), s_p1.get(0, G.ci(cx, cy + 1)),
                           s_phi.get(s0, G.ci(cx, cy)), s_phi.get(s0, G.ci(cx, cy + 1)), dph);
              {
                lds_face_tangential<R, 1>(s_phi, G, cx, cy, sm, s0, sp, inv_4dx, gt1, gt2);
                mu_face_j<R, false>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
              }
            }
            s_fy[0][fo] = Phi[0];
            s_fy[1][fo] = Phi[1];
          }
        }
        // z face above plane k
        if (g.zface(k)) {
          R pb[NP], gn[NP];
          lds_face_normal<R, 2>(s_phi, G, G.lx + 1, G.ly + 1, s0, sp, inv_dx, pb, gn);
          mu_face_diff<R, true>(P, C, pb, ownm, upm, Pzu);
          if (antitrap && mu_face_needs_j(pb)) {
            R gt1[NP], gt2[NP], dph[3];
            const V4<R> L0 = s_phi.get(s0, G.own_c), U0 = s_phi.get(sp, G.own_c);
  #pragma unroll
            for (int a = 0; a < 3; ++a) dph[a] = (own1.v[a] - L0.v[a]) + (up1.v[a] - U0.v[a]);
            {
              lds_face_tangential<R, 2>(s_phi, G, G.lx + 1, G.ly + 1, sm, s0, sp, inv_4dx, gt1, gt2);
              mu_face_j<R, true>(P, C, pb, gn, gt1, gt2, dph, ownm, upm, Pzu);
            }
          }
        }
      }
      V4<R> own0;
      if (cells) own0 = s_phi.get(s0, G.own_c);
      __syncthreads();  // B1: faces visible; phi slot of k-1 and mu plane k free
      {
        const int sl = slot_of(NSLOT, k + AHEAD);
        s_phi.put(sl, G.own_c, nxt_own);
        if (G.halo_c >= 0) s_phi.put(sl, G.halo_c, nxt_halo);
        s_mu.put(G.own_c, upm);
        if (G.halo_c >= 0) s_mu.put(G.halo_c, nxt_hm);
        s_p1.put(0, G.own_c, up1);
        if (G.halo_c >= 0) s_p1.put(0, G.halo_c, nxt_p1h);
      }
      if (cells && G.valid) {
        const int fl = G.ly * (G.tx + 1) + G.lx;
        const int yl = G.ly * G.tx + G.lx;
        R div[NM], out[NM];
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          div[q] = R(0);
          div[q] += s_fx[q][fl + 1] - s_fx[q][fl];
          div[q] += s_fy[q][yl + G.tx] - s_fy[q][yl];
          div[q] = (div[q] + (Pzu[q] - Pzl[q])) * inv_dx;
        }
        mu_cell<R>(P, C, own0.v, own1.v, ownm, div, out);
        stg<R>(dst.at(4, k), G.own_b, out[0]);
        stg<R>(dst.at(5, k), G.own_b, out[1]);
      }
      Pzl[0] = Pzu[0];
      Pzl[1] = Pzu[1];
      own1 = up1;
      ownm[0] = upm[0];
      ownm[1] = upm[1];
      __syncthreads();  // B2
    }
  }
}

// The FP32 instance is held to 128 VGPRs so that four waves fit per SIMD.
__global__ __launch_bounds__(kTileThreads) void mu_tiled_f64(DevDomain* const* doms, const int32_t* first,
                                                             int ndom, int total, const uint32_t* words) {
  mu_tiled_body<double>(doms, first, ndom, total, words);
}
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(4))) void mu_tiled_f32(
    DevDomain* const* doms, const int32_t* first, int ndom, int total, const uint32_t* words) {
  mu_tiled_body<float>(doms, first, ndom, total, words);
}

// mu-sweep of the items whose faces carry no anti-trapping current
// (item_jfree): only the diffusive fluxes M grad mu, which need phi^n at
// the face cells (one LDS plane and the own column in registers, as in the
// isotropic phi-sweep) and mu^n; no tangential gradients and no phi^{n+1}
// neighbours.  Every face value and the cell stage are the same operations
// on the same operands as in mu_tiled_body, so both kernels give bitwise
// the same mu^{n+1} on such an item.
// The LDS of the light items' body.
template <typename R>
struct BulkLds {
  LdsPhi<R, 1> phi;  // phi^n of plane k
  LdsMu<R> mu;       // mu^n of plane k
  R fx[NM][kMaxFx];
  R fy[NM][kFyCap<R>];
};

template <typename R>
__device__ __forceinline__ void mu_bulk_item(const ItemCtx<R>& X, BulkLds<R>& L, int t) {
  LdsPhi<R, 1>& s_phi = L.phi;
  LdsMu<R>& s_mu = L.mu;
  R (*s_fx)[kMaxFx] = L.fx;
  R (*s_fy)[kFyCap<R>] = L.fy;
  const int wave = t >> 6, lane = t & 63;
  {
    const TileGeo& G = X.G;
    const Geo& g = X.g;
    const auto& P = kparams<R>(*X.dp);
    const Copy& src = X.src;  // phi^n (fields 0-3), mu^n (4-5)
    const Copy& dst = X.dst;  // phi^{n+1}, mu^{n+1}
    const R inv_dx = (R)P.inv_dx;
    __syncthreads();  // the previous item's LDS is consumed (it may be a pure item's)
    const bool ex_ok = lane < G.ty && G.y0 + lane < g.ny;
    const bool ey_ok = lane < G.tx && G.x0 + lane < g.nx;
    const int kstart = G.z0 - 1;

    const int kc0 = g.zc(kstart);
    V4<R> own_k = load4<R>(src, kc0, G.own_b);
    R ownm[NM] = {ldg<R>(src.at(4, kc0), G.own_b), ldg<R>(src.at(5, kc0), G.own_b)};
    s_phi.put(0, G.own_c, own_k);
    s_mu.put(G.own_c, ownm);
    if (G.halo_c >= 0) {
      s_phi.put(0, G.halo_c, load4<R>(src, kc0, G.halo_b));
      const R hm[NM] = {ldg<R>(src.at(4, kc0), G.halo_b), ldg<R>(src.at(5, kc0), G.halo_b)};
      s_mu.put(G.halo_c, hm);
    }
    __syncthreads();

    R Pzl[NM] = {R(0), R(0)};
    for (int k = kstart; k < G.z1; ++k) {
      const bool cells = k >= G.z0;
      // plane k+1 (phi^n, mu^n: own column and halo cell), then phi^{n+1}
      // of the own cell at plane k (cell stage only)
      const int k1 = g.zp(k);
      const V4<R> nxt_own = load4<R>(src, k1, G.own_b);
      const R upm[NM] = {ldg<R>(src.at(4, k1), G.own_b), ldg<R>(src.at(5, k1), G.own_b)};
      V4<R> nxt_halo;
      R nxt_hm[NM] = {R(0), R(0)};
      if (G.halo_c >= 0) {
        nxt_halo = load4<R>(src, k1, G.halo_b);
        nxt_hm[0] = ldg<R>(src.at(4, k1), G.halo_b);
        nxt_hm[1] = ldg<R>(src.at(5, k1), G.halo_b);
      }
      V4<R> own1;
      if (cells && G.valid) own1 = load4<R>(dst, k, G.own_b);
      const int kk = k < 0 ? 0 : k;
      const auto& C = X.tab[kk];
      if (cells) {
        const bool ex = ex_ok && wave == ((k + 1) & 3);
        const bool ey = ey_ok && wave == (k & 3);
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          const bool edge = r == 1;
          if (edge ? !ex : !G.valid) continue;
          const int cx = edge ? 0 : G.lx + 1, cy = edge ? lane + 1 : G.ly + 1;
          const int fo = edge ? lane * (G.tx + 1) : G.ly * (G.tx + 1) + G.lx + 1;
          R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
          lds_face_normal<R, 0>(s_phi, G, cx, cy, 0, 0, inv_dx, pb, gn);
          s_mu.get(G.ci(cx, cy), mL);
          s_mu.get(G.ci(cx + 1, cy), mU);
          mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
          s_fx[0][fo] = Phi[0];
          s_fx[1][fo] = Phi[1];
        }
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          const bool edge = r == 1;
          if (edge ? !ey : !G.valid) continue;
          const int cx = edge ? lane + 1 : G.lx + 1, cy = edge ? 0 : G.ly + 1;
          const int fo = edge ? lane : (G.ly + 1) * G.tx + G.lx;
          R pb[NP], gn[NP], mL[NM], mU[NM], Phi[NM];
          lds_face_normal<R, 1>(s_phi, G, cx, cy, 0, 0, inv_dx, pb, gn);
          s_mu.get(G.ci(cx, cy), mL);
          s_mu.get(G.ci(cx, cy + 1), mU);
          mu_face_diff<R, false>(P, C, pb, mL, mU, Phi);
          s_fy[0][fo] = Phi[0];
          s_fy[1][fo] = Phi[1];
        }
      }
      // z face above plane k: own column at k and k+1
      R Pzu[NM] = {R(0), R(0)};
      if (g.zface(k)) {
        R pb[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) pb[a] = R(0.5) * (own_k.v[a] + nxt_own.v[a]);
        mu_face_diff<R, true>(P, C, pb, ownm, upm, Pzu);
      }
      __syncthreads();  // B1: faces visible; phi and mu planes of k free
      s_phi.put(0, G.own_c, nxt_own);
      s_mu.put(G.own_c, upm);
      if (G.halo_c >= 0) {
        s_phi.put(0, G.halo_c, nxt_halo);
        s_mu.put(G.halo_c, nxt_hm);
      }
      if (cells && G.valid) {
        const int fl = G.ly * (G.tx + 1) + G.lx;
        const int yl = G.ly * G.tx + G.lx;
        R div[NM], out[NM];
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          div[q] = R(0);
          div[q] += s_fx[q][fl + 1] - s_fx[q][fl];
          div[q] += s_fy[q][yl + G.tx] - s_fy[q][yl];
          div[q] = (div[q] + (Pzu[q] - Pzl[q])) * inv_dx;
        }
        mu_cell<R>(P, C, own_k.v, own1.v, ownm, div, out);
        stg<R>(dst.at(4, k), G.own_b, out[0]);
        stg<R>(dst.at(5, k), G.own_b, out[1]);
      }
      Pzl[0] = Pzu[0];
      Pzl[1] = Pzu[1];
      own_k = nxt_own;
      ownm[0] = upm[0];
      ownm[1] = upm[1];
      __syncthreads();  // B2: LDS planes and faces consumed
    }
  }
}



// The coefficients of one plane that a cell pure in phase a uses, in the
// order mu_pure_item stages them, two components each: Mp, MpZ, rchip, and
// dchi, dcbar of phase a.
constexpr int kPureCoef = 5 * NM;
template <typename R>
__device__ __forceinline__ R pure_coef(const PF_CONST PlaneCoef<R>& C, int a, int j) {
  const int q = j & 1;
  switch (j >> 1) {
    case 0: return C.Mp[a][q];
    case 1: return C.MpZ[a][q];
    case 2: return C.rchip[a][q];
    case 3: return C.dchi[a][q];
    default: return C.dcbar[a][q];
  }
}

// mu-sweep of the items that mu_pure_phase finds pure in phase a: phi^n =
// phi^{n+1} = e_a on every cell read, so a thread needs only mu^n of its
// column and of its four lateral neighbours (the latter from an LDS plane
// that the own columns and the halo ring fill).
//
// Same result as the other bodies, operation by operation: each face flux
// is mu_face_flux of the same two mu values with the coefficient M that
// mu_face_m gives at pb = e_a (the plane's Mp, MpZ, computed by that
// function); the divergence sums the fluxes in the same order; in mu_cell
// at phi^n = phi^{n+1} = e_a, h = e_a exactly and h1 - h0 = +0, so every
// term of the src sum but one multiplies a finite value by +0 and adds a
// zero: src is fma_(h_a, ta_a, +0), which is what the full sum gives (a
// zero sum stays +0 before and after that term); the chi sum's reciprocal
// is the plane's rchip.  For every finite state mu^{n+1} is bitwise the
// other bodies', from a third of the bytes and a quarter of the arithmetic.

// Planes of mu^n each thread of mu_pure_item has in flight ahead of the
// one it evaluates.
constexpr int kPureAhead = 4;

// The LDS of the pure items' body.
// Planes of the pure-item body per barrier: FP64 two (four plane buffers
// keep mu_light_f64's LDS within its light body's), FP32 four.
template <typename R>
constexpr int kPureGroup = sizeof(R) == 8 ? 2 : 4;
template <typename R>
struct PureLds {
  LdsMu<R> m[2 * kPureGroup<R>];  // mu^n with the halo ring, two groups of planes
  R cf[kMaxZc][kPureCoef];  // the item's plane coefficients, staged once (the
                            // table is too large for the scalar cache, and a
                            // scalar load per value and plane would put a round
                            // trip to L2 into every plane)
};

// The pure-item test of the mu-sweep for this item, or -1; a pure item is
// counted and marked (kMuPure) for the other mu kernels of the step.
template <typename R>
__device__ __forceinline__ int mu_pure_take(const ItemCtx<R>& X, int t) {
  const auto& P = kparams<R>(*X.dp);
  if (!P.shortcuts || P.mu_frozen) return -1;  // uniform
  const int a = mu_pure_phase(*X.dp, chunk_id(*X.dp, X.G));
  if (a >= 0 && t == 0) {
    atomicAdd(X.jc + count_word(kCountPure, X.slot), 1u);
    // for the other mu kernels of the step (the phi-sweep rewrote the word)
    *to_global(X.jf) = *to_const(X.jf) | kMuPure;
  }
  return a;  // uniform
}

template <typename R>
__device__ __forceinline__ void mu_pure_item(const ItemCtx<R>& X, int a, PureLds<R>& L, int t) {
  R (*s_cf)[kPureCoef] = L.cf;
  LdsMu<R>* s_m = L.m;
  const auto& P = kparams<R>(*X.dp);
  {
    const TileGeo& G = X.G;
    const Geo& g = X.g;
    const Copy& src = X.src;
    const Copy& dst = X.dst;
    const R inv_dx = (R)P.inv_dx;
    const int z0 = G.z0, z1 = G.z1;
    __syncthreads();  // the previous item's LDS planes and coefficients are consumed
    for (int i = t; i < (z1 - z0) * kPureCoef; i += blockDim.x)
      s_cf[i / kPureCoef][i % kPureCoef] = pure_coef<R>(X.tab[z0 + i / kPureCoef], a, i % kPureCoef);
    R ha;  // h_a of a cell holding e_a (1)
    {
      R e[NP], h[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) e[b] = b == a ? R(1) : R(0);
      mu_cell_h<R>(e, h);
      ha = h[a];
    }
    // Ring of mu^n loads, slot p % kPureAhead for plane p: the own column
    // for planes z0 .. z1 (plane z1 feeds the z face above the last plane;
    // zc gives the mirror or the ghost plane there) and this thread's halo
    // cell for planes z0 .. z1-1.  Only these loads go to global memory, so
    // a wait for plane k's values never waits for the loads issued after
    // them (the memory counter is in order).  The loads are unconditional:
    // past the item's planes they read its last needed plane again (a cache
    // hit, not another plane from memory), and a thread without a halo cell
    // reads its own column again; a load on only some paths made the
    // compiler move its value between registers, waiting for it at once.
    // The four corners of the halo ring are not read (the stencil here has
    // no tangential part), so their threads take no halo cell either.
    R ro[kPureAhead][NM], rh[kPureAhead][NM];
    const bool corner = t == 0 || t == G.tx + 1 || t == G.tx + 2 || t == 2 * G.tx + 3;
    const bool halo = G.halo_c >= 0 && !corner;
    const uint32_t hb = halo ? G.halo_b : G.own_b;
    const auto fetch = [&](int p, R o[NM], R hv[NM]) {
      const int pc = g.zc(p < z1 ? p : z1), ph = g.zc(p < z1 ? p : z1 - 1);
      o[0] = ldg<R>(src.at(4, pc), G.own_b);
      o[1] = ldg<R>(src.at(5, pc), G.own_b);
      hv[0] = ldg<R>(src.at(4, ph), hb);
      hv[1] = ldg<R>(src.at(5, ph), hb);
    };
#pragma unroll
    for (int u = 0; u < kPureAhead; ++u) fetch(z0 + u, ro[u], rh[u]);
    // the z face below z0 as the sweep of the plane below evaluates it
    R Pzl[NM] = {R(0), R(0)};
    const int kb = z0 - 1;
    if (g.zface(kb)) {
      const R mb[NM] = {ldg<R>(src.at(4, g.zc(kb)), G.own_b), ldg<R>(src.at(5, g.zc(kb)), G.own_b)};
#pragma unroll
      for (int q = 0; q < NM; ++q)
        Pzl[q] = mu_face_flux<R>(X.tab[kb].MpZ[a][q], mb[q], ro[0][q], inv_dx);
    }
    const int ox = G.lx + 1, oy = G.ly + 1;
    // planes in groups of Gp: all go to LDS before one barrier; the groups
    // alternate between two halves of the buffers, so a group writes the
    // half whose reads (two groups back) ended before the last barrier
    constexpr int Gp = kPureGroup<R>;
    static_assert(kPureAhead % Gp == 0, "groups of ring slots");
    const auto plane = [&](int k, const LdsMu<R>& sm, const R m[NM], const R up[NM]) {
      if (!G.valid) return;
      const R* cf = s_cf[k - z0];
      const bool zf = g.zface(k);
      R L[4][NM];
      sm.get(G.ci(ox - 1, oy), L[0]);
      sm.get(G.ci(ox + 1, oy), L[1]);
      sm.get(G.ci(ox, oy - 1), L[2]);
      sm.get(G.ci(ox, oy + 1), L[3]);
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        const R Mxy = cf[q];
        const R fxl = mu_face_flux<R>(Mxy, L[0][q], m[q], inv_dx);
        const R fxu = mu_face_flux<R>(Mxy, m[q], L[1][q], inv_dx);
        const R fyl = mu_face_flux<R>(Mxy, L[2][q], m[q], inv_dx);
        const R fyu = mu_face_flux<R>(Mxy, m[q], L[3][q], inv_dx);
        const R Pzu = zf ? mu_face_flux<R>(cf[2 + q], m[q], up[q], inv_dx) : R(0);
        R div = R(0);
        div += fxu - fxl;
        div += fyu - fyl;
        div = (div + (Pzu - Pzl[q])) * inv_dx;
        Pzl[q] = Pzu;
        const R sq = mu_pure_src<R>(ha, cf[6 + q], cf[8 + q], m[q]);
        stg<R>(dst.at(4 + q, k), G.own_b, mu_cell_out<R>(P, div, sq, cf[4 + q], m[q]));
      }
    };
    for (int k0 = z0; k0 < z1; k0 += kPureAhead) {
#pragma unroll
      for (int u = 0; u < kPureAhead; u += Gp) {
        const int k = k0 + u;
        if (k >= z1) break;  // uniform
        // buffers of this group: the two halves alternate from group to group
        LdsMu<R>* sb = s_m + (((k - z0) / Gp) & 1) * Gp;
        // planes k .. k+Gp-1 into LDS; their own values and the ones above
        // in registers (constant slots once unrolled)
        R mv[Gp + 1][NM];
#pragma unroll
        for (int j = 0; j < Gp; ++j) {
          mv[j][0] = ro[u + j][0];
          mv[j][1] = ro[u + j][1];
        }
#pragma unroll
        for (int j = 0; j < Gp; ++j) {
          if (k + j >= z1) break;  // uniform
          sb[j].put(G.own_c, mv[j]);
          if (halo) sb[j].put(G.halo_c, rh[u + j]);
        }
        // the group's slots are free: planes kPureAhead further on
#pragma unroll
        for (int j = 0; j < Gp; ++j) fetch(k + j + kPureAhead, ro[u + j], rh[u + j]);
        // plane k+Gp, above the group's last plane: still in the ring when
        // the group is shorter than the ring, else the load just issued
        mv[Gp][0] = ro[(u + Gp) % kPureAhead][0];
        mv[Gp][1] = ro[(u + Gp) % kPureAhead][1];
        __syncthreads();  // the group's planes visible
#pragma unroll
        for (int j = 0; j < Gp; ++j) {
          if (k + j >= z1) break;  // uniform
          plane(k + j, sb[j], mv[j], mv[j + 1]);
        }
      }
    }
  }
}

// FP32: the pure items (mu_tiled_f32 takes the rest).
__global__ __launch_bounds__(kTileThreads) void mu_pure_f32(DevDomain* const* doms, const int32_t* first,
                                                            int ndom, int total) {
  __shared__ PureLds<float> L;
  const int t = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    ItemCtx<float> X;
    if (!item_setup(doms, first, ndom, item, t, X)) continue;
    const int a = mu_pure_take(X, t);
    if (a >= 0) mu_pure_item(X, a, L, t);
  }
}

// FP64: the pure items, and the light items when the split runs
// (mu_tiled_f64 takes the rest).  One launch for both, so that the few
// long light items overlap the many pure ones; they share the LDS, one item
// at a time.
__global__ __launch_bounds__(kTileThreads) void mu_light_f64(DevDomain* const* doms, const int32_t* first,
                                                             int ndom, int total) {
  constexpr size_t kB = sizeof(BulkLds<double>), kP = sizeof(PureLds<double>);
  __shared__ __align__(16) unsigned char smem[kB > kP ? kB : kP];
  const int t = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    ItemCtx<double> X;
    if (!item_setup(doms, first, ndom, item, t, X)) continue;
    const int a = mu_pure_take(X, t);
    if (a >= 0) {
      mu_pure_item(X, a, *reinterpret_cast<PureLds<double>*>(smem), t);
    } else if (item_light(*X.dp, X)) {
      mu_bulk_item(X, *reinterpret_cast<BulkLds<double>*>(smem), t);
    }
  }
}

// --------------------------------------------------------------- launches

// The copy that does not hold the state has been overwritten (staging of a
// host read or a checkpoint): no chunk is held by both copies any more.
__global__ __launch_bounds__(256) void drop_same_kernel(uint8_t* flags, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = (uint8_t)(flags[i] & ~kSame);
}

hipError_t launch_drop_same(uint8_t* flags, int64_t n, hipStream_t s) {
  const int64_t b = (n + 255) / 256;
  drop_same_kernel<<<(int)(b < 1024 ? (b > 0 ? b : 1) : 1024), 256, 0, s>>>(flags, n);
  return hipGetLastError();
}

hipError_t launch_phi_tiled(const LaunchSet& L, int prec, bool aniso, hipStream_t s) {
  const int grid = L.total;
  const int per = bulk_items_per_wave(L.total);
  if (prec == 0)
    phi_bulk_kernel<double><<<(grid + per * kTileWaves - 1) / (per * kTileWaves), kTileThreads, 0, s>>>(
        L.doms, L.first, L.ndom, L.total, per);
  else
    phi_bulk_kernel<float><<<(grid + per * kTileWaves - 1) / (per * kTileWaves), kTileThreads, 0, s>>>(
        L.doms, L.first, L.ndom, L.total, per);
  if (prec == 0) {
    if (aniso)
      phi_tiled_f64_aniso<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
    else
      phi_tiled_f64<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
  } else {
    if (aniso)
      phi_tiled_f32_aniso<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
    else
      phi_tiled_f32<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
  }
  return hipGetLastError();
}

// The mu-sweep launches over the same items.  FP64: mu_light_f64 takes the
// items pure in one phase, and the light items when they are the large
// majority; mu_tiled_f64 the rest.  FP32: mu_pure_f32 takes the pure items,
// mu_tiled_f32 the rest.
hipError_t launch_mu_tiled(const LaunchSet& L, int prec, hipStream_t s) {
  const int grid = L.total;
  if (prec == 0) {
    mu_light_f64<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
    mu_tiled_f64<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
  } else {
    mu_pure_f32<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
    mu_tiled_f32<<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total, L.words);
  }
  return hipGetLastError();
}

}  // namespace pfk
