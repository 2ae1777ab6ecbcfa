// pf_runtime.hip -- host runtime behind the C ABI declared in pfsolve.h.
//
// Owns the device layout of a domain (one allocation: descriptor, work-item
// table, per-plane coefficient table, diagnostics scratch, Voronoi phase map,
// and two copies of the six fields phi_0..3, mu_0..1, structure of arrays,
// x fastest, rows padded to 128 bytes), validates parameters, resolves the
// time step, and enqueues the kernels of Algorithm 1 on the domain's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pfsolve.h"
#include "pf_device.h"
#include "pf_launch.h"

using namespace pfk;

namespace {

thread_local std::string g_last_error;
std::atomic<int> g_variant{1};

pf_status fail(pf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define PF_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PF_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Tiling {
  int32_t tx, ty, zc, ntx, nty, nzc;
  int32_t xmode, rs;  // XCD y-slab order and tile rows per XCD
  // blocks of one launch over this domain: a multiple of 8 so that a
  // domain's first block sits on XCD 0 in a pack as well
  int32_t blocks() const {
    if (xmode) return 8 * rs * ntx * nzc;
    return (ntx * nty * nzc + 7) / 8 * 8;
  }
};

Tiling choose_tiling(int nx, int ny, int nz, int prec) {
  Tiling t;
  t.tx = nx >= 48 && prec != PF_FP64 ? 64 : 32;
  t.ty = kTileThreads / t.tx;
  t.ntx = (nx + t.tx - 1) / t.tx;
  t.nty = (ny + t.ty - 1) / t.ty;
  // z chunk: 32 planes, fewer (down to 8) while that leaves fewer than
  // ~2048 work items.  Long chunks let neighbouring tiles drift apart in z,
  // so the halo cells one tile loads are evicted from L2 before its
  // neighbour reads them; short ones re-load more ring planes.
  const int64_t cols = (int64_t)nz * t.ntx * t.nty;
  const int64_t zc = std::min<int64_t>(kMaxZc, std::max<int64_t>(8, cols / 2048));
  t.zc = (int32_t)std::min<int64_t>(zc, nz);
  t.nzc = (nz + t.zc - 1) / t.zc;
  // y-slab order when it leaves at most 1/8 of the blocks without a tile
  t.rs = (t.nty + 7) / 8;
  t.xmode = (8 * t.rs - t.nty) * 8 <= 8 * t.rs ? 1 : 0;
  return t;
}

struct Layout {
  int32_t pitch;
  int64_t plane, fstride;  // elements
  size_t elem;
  size_t off_desc, off_ptrs, off_first, off_coef, off_jfree, off_pflag, off_mesh, off_partials,
      off_diag, off_map, off_fields;
  size_t pflag_bytes;
  size_t copy_bytes, total;
};

bool make_layout(const pf_domain_desc& d, Layout& L) {
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return false;
  if (d.prec != PF_FP64 && d.prec != PF_FP32) return false;
  if (!(d.dx > 0.0) || !std::isfinite(d.dx)) return false;
  L.elem = d.prec == PF_FP64 ? 8 : 4;
  const int64_t row_elems = 128 / (int64_t)L.elem;
  const int64_t pitch = (d.nx + row_elems - 1) / row_elems * row_elems;
  if (pitch > INT32_MAX) return false;
  // the tiled sweeps address a cell within its field plane by a 32-bit byte
  // offset: a plane (pitch x ny elements) must stay below 4 GiB
  if ((uint64_t)pitch * (uint64_t)d.ny * L.elem > (uint64_t)UINT32_MAX) return false;
  L.pitch = (int32_t)pitch;
  const long double cells = (long double)pitch * d.ny * d.nz;
  if (cells * L.elem * 12 > (long double)(1ull << 62)) return false;
  {  // work items of the tiled sweeps must fit the 32-bit block index
    const int64_t tx = d.nx >= 48 && d.prec != PF_FP64 ? 64 : 32, ty = kTileThreads / tx;
    const int64_t items = ((d.nx + tx - 1) / tx) * ((d.ny + ty - 1) / ty) * (int64_t)d.nz;
    if (items > (int64_t)1 << 28) return false;
  }
  L.plane = pitch * (int64_t)d.ny;
  // fields start 4 KiB apart plus a 2 KiB skew, so that equal offsets in
  // different fields do not fall on the same memory channel; each field has
  // nz + 1 planes, the last being the ghost plane of a Dirichlet top
  const int64_t fe = L.plane * ((int64_t)d.nz + 1);
  const int64_t a4k = 4096 / (int64_t)L.elem, skew = 2048 / (int64_t)L.elem;
  L.fstride = (fe + a4k - 1) / a4k * a4k + skew;
  size_t off = 0;
  L.off_desc = off;
  off = align_up(off + sizeof(DevDomain), kAlign);
  L.off_ptrs = off;
  off = align_up(off + sizeof(void*), kAlign);
  L.off_first = off;
  off = align_up(off + 2 * sizeof(int32_t), kAlign);
  L.off_coef = off;
  const size_t coef_sz = d.prec == PF_FP64 ? sizeof(PlaneCoef<double>) : sizeof(PlaneCoef<float>);
  off = align_up(off + coef_sz * (size_t)d.nz, kAlign);
  const Tiling T = choose_tiling(d.nx, d.ny, d.nz, d.prec);
  L.off_jfree = off;  // one 32-bit word per work item of the tiled sweeps, then the counts
  off = align_up(off + sizeof(uint32_t) * ((size_t)count_base(T.blocks()) + kCountWords), kAlign);
  L.pflag_bytes = align_up((size_t)T.ntx * T.nty * T.nzc, kAlign);
  L.off_pflag = off;  // the pure-phase flags of each copy's state, then those of the
  off += 4 * L.pflag_bytes;  // chunks' end planes
  L.off_mesh = off;  // triangle counter of pf_mesh_phase
  off = align_up(off + sizeof(unsigned long long), kAlign);
  L.off_partials = off;
  off = align_up(off + sizeof(double) * kDiagBlocks * kDiagValues, kAlign);
  L.off_diag = off;
  off = align_up(off + sizeof(double) * kDiagValues, kAlign);
  L.off_map = off;
  off = align_up(off + (size_t)d.nx * (size_t)d.ny, 4096);
  L.off_fields = off;
  L.copy_bytes = align_up((size_t)L.fstride * NFIELD * L.elem, 4096);
  L.total = off + 2 * L.copy_bytes;
  return true;
}

uint64_t splitmix64_next(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Column -> solid phase map of the Voronoi initial state (2D).
void voronoi_columns(int nx, int ny, uint64_t seed, int nseeds, std::vector<int8_t>& map) {
  map.assign((size_t)nx * ny, (int8_t)LQ);
  if (nseeds <= 0) return;
  std::vector<double> sx(nseeds), sy(nseeds);
  uint64_t st = seed;
  for (int s = 0; s < nseeds; ++s) {
    sx[s] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 * nx;
    sy[s] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 * ny;
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double cx = (double)i + 0.5, cy = (double)j + 0.5;
      double best_d = INFINITY;
      int best = 0;
      for (int s = 0; s < nseeds; ++s) {
        double ax = std::fabs(cx - sx[s]), ay = std::fabs(cy - sy[s]);
        if (nx - ax < ax) ax = nx - ax;
        if (ny - ay < ay) ay = ny - ay;
        const double d2 = ax * ax + ay * ay;
        if (d2 < best_d) {
          best_d = d2;
          best = s;
        }
      }
      map[(size_t)j * nx + i] = (int8_t)(best % 3);
    }
}

}  // namespace

struct pf_domain {
  pf_domain_desc desc;
  Layout L;
  Tiling T;
  char* base = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  DevDomain host;  // host mirror of the descriptor's static part
  DevDomain* dev = nullptr;
  DevDomain** dev_ptrs = nullptr;
  int32_t* dev_first = nullptr;
  bool params_set = false, fields_set = false, aniso = false;
  double dt = 0.0, bound = 0.0;
  int32_t diag_every = 0;
  int64_t since_diag = 0;
  bool diag_pending = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> timing_events;
  pf_pack* pack = nullptr;
  hipStream_t pack_stream = nullptr;  // stream of the pack this domain belongs to

  char* fields(int copy) const { return base + L.off_fields + (size_t)copy * L.copy_bytes; }
  double* partials() const { return reinterpret_cast<double*>(base + L.off_partials); }
  double* diag_out() const { return reinterpret_cast<double*>(base + L.off_diag); }
  LaunchSet launch_set() const {
    LaunchSet s;
    s.doms = dev_ptrs;
    s.first = dev_first;
    s.ndom = 1;
    s.total = T.blocks();
    s.words = reinterpret_cast<const uint32_t*>(base + L.off_jfree);
    return s;
  }
};

namespace {

pf_status upload_desc(pf_domain* d) {
  PF_HIP(hipMemcpyAsync(d->dev, &d->host, sizeof(DevDomain), hipMemcpyHostToDevice, d->stream));
  return PF_OK;
}

// Wait for the domain's own stream and, for a pack member, the pack's.
pf_status sync_domain(pf_domain* d) {
  PF_HIP(hipStreamSynchronize(d->stream));
  if (d->pack) PF_HIP(hipStreamSynchronize(d->pack_stream));
  return PF_OK;
}

// Read the device descriptor's dynamic state (step, parity, steps left).
pf_status fetch_state(pf_domain* d, DevDomain& out) {
  pf_status st = sync_domain(d);
  if (st != PF_OK) return st;
  PF_HIP(hipMemcpyAsync(&out, d->dev, sizeof(DevDomain), hipMemcpyDeviceToHost, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  return PF_OK;
}

double temperature(const pf_params& p, double z, double t) {
  return p.T0 + p.G * (z + p.zoff - p.v * t);
}

pf_status validate_and_bound(const pf_domain* d, const pf_params& p, double& bound) {
  const double dx = d->desc.dx;
  if (!(p.eps > 0.0) || !std::isfinite(p.eps)) return fail(PF_ERR_INVALID_ARG, "eps must be > 0");
  double tau_min = INFINITY, gmax = 0.0, dmax = 0.0;
  for (int a = 0; a < NP; ++a) {
    if (!(p.tau[a] > 0.0)) return fail(PF_ERR_INVALID_ARG, "tau must be > 0");
    if (!(p.D[a] >= 0.0)) return fail(PF_ERR_INVALID_ARG, "D must be >= 0");
    tau_min = std::min(tau_min, p.tau[a]);
    for (int b = 0; b < NP; ++b) {
      if (a == b) continue;
      if (!(p.gamma[a][b] >= 0.0) || p.gamma[a][b] != p.gamma[b][a])
        return fail(PF_ERR_INVALID_ARG, "gamma must be symmetric and >= 0");
      if (!(p.aniso_delta[a][b] >= 0.0) || !(p.aniso_delta[a][b] < 1.0 / 15.0) ||
          p.aniso_delta[a][b] != p.aniso_delta[b][a])
        return fail(PF_ERR_INVALID_ARG, "anisotropy delta must be symmetric and in [0, 1/15)");
      gmax = std::max(gmax, p.gamma[a][b]);
      dmax = std::max(dmax, p.aniso_delta[a][b]);
    }
  }
  if (!(p.gamma3 >= 0.0)) return fail(PF_ERR_INVALID_ARG, "gamma3 must be >= 0");
  const double Tb = temperature(p, 0.0, 0.0);
  const double Tt = temperature(p, (double)(d->desc.nz - 1) * dx, 0.0);
  const double Tmax = std::max(Tb, Tt), Tmin = std::min(Tb, Tt);
  if (!(Tmin > 0.0)) return fail(PF_ERR_INVALID_ARG, "temperature must be > 0 over the domain");
  double chi_min = INFINITY, dchi_max = 0.0;
  for (int a = 0; a < NP; ++a)
    for (int q = 0; q < NM; ++q)
      for (double T : {Tmin, Tmax}) {
        const double c = p.chi0[a][q] + p.chi1[a][q] * (T - p.TE);
        if (!(c > 0.0)) return fail(PF_ERR_INVALID_ARG, "susceptibility must be > 0");
        chi_min = std::min(chi_min, c);
        dchi_max = std::max(dchi_max, p.D[a] * c);
      }
  // phase field: two-phase diffusivity 2 gamma T / tau, 7-point limit
  // dx^2/(6 D), cubic stiffening (1+delta)(1+15 delta)
  const double kappa = (1.0 + dmax) * (1.0 + 15.0 * dmax);
  const double dt_phi = gmax > 0.0 ? dx * dx * tau_min / (12.0 * gmax * Tmax * kappa) : INFINITY;
  const double dt_mu = dchi_max > 0.0 ? dx * dx * chi_min / (6.0 * dchi_max) : INFINITY;
  bound = std::min(dt_phi, dt_mu);
  if (!std::isfinite(bound)) return fail(PF_ERR_INVALID_ARG, "no finite stability bound");
  return PF_OK;
}

template <typename R>
void fill_kparams(KParams<R>& k, const pf_params& p, double dt, double dx, bool aniso) {
  const double pi = 3.14159265358979323846;
  for (int a = 0; a < NP; ++a)
    for (int b = a + 1; b < NP; ++b) {
      const int i = pair_index(a, b);
      k.g1[i] = (R)p.gamma[a][b];
      k.g2[i] = (R)(2.0 * p.gamma[a][b]);
      k.g16[i] = (R)(16.0 / (pi * pi) * p.gamma[a][b]);
      k.delta[i] = (R)p.aniso_delta[a][b];
      k.ac0[i] = (R)(1.0 - 3.0 * p.aniso_delta[a][b]);
      k.d4[i] = (R)(4.0 * p.aniso_delta[a][b]);
      k.d16[i] = (R)(16.0 * p.aniso_delta[a][b]);
    }
  k.gamma3 = (R)p.gamma3;
  for (int a = 0; a < NP; ++a) k.rate[a] = (R)(dt / (p.tau[a] * p.eps));
  k.inv_dx = (R)(1.0 / dx);
  k.inv_4dx = (R)(1.0 / (4.0 * dx));
  k.dt = (R)dt;
  k.half_inv_dt = (R)(0.5 / dt);
  k.pieps4 = (R)(pi * p.eps / 4.0);
  k.aniso = aniso ? 1 : 0;
  k.antitrap = p.antitrapping ? 1 : 0;
  k.mu_frozen = p.mu_frozen ? 1 : 0;
  k.shortcuts = p.shortcuts ? 1 : 0;
  k.aniso_mask = 0;
  for (int a = 0; a < NP; ++a)
    for (int b = a + 1; b < NP; ++b)
      if (p.aniso_delta[a][b] > 0.0) k.aniso_mask |= 1 << pair_index(a, b);
  k.pad[0] = k.pad[1] = k.pad[2] = 0;
}

pf_status enqueue_step(pf_domain* d, hipEvent_t* ev) {
  const LaunchSet s = d->launch_set();
  const int prec = d->desc.prec;
  const int var = g_variant.load();
  PF_HIP(launch_prologue(s, prec, d->stream));
  if (d->host.window_z > 0) PF_HIP(launch_window(s, prec, d->stream));
  if (ev) PF_HIP(hipEventRecord(ev[0], d->stream));
  PF_HIP(launch_phi(s, prec, d->aniso, var, d->stream));
  if (ev) PF_HIP(hipEventRecord(ev[1], d->stream));
  PF_HIP(launch_mu(s, prec, var, d->stream));
  if (ev) PF_HIP(hipEventRecord(ev[2], d->stream));
  return PF_OK;
}

pf_status check_state(const pf_domain* d) {
  if (!d) return fail(PF_ERR_INVALID_ARG, "null domain");
  if (!d->params_set) return fail(PF_ERR_STATE, "pf_set_params has not been called");
  if (!d->fields_set) return fail(PF_ERR_STATE, "pf_init_fields has not been called");
  return PF_OK;
}

pf_status run_diag(pf_domain* d, double t, double out[kDiagValues]) {
  PF_HIP(launch_diag(d->dev, d->desc.prec, d->desc.nx, d->desc.ny, d->desc.nz, t, d->partials(),
                     d->diag_out(), d->stream));
  PF_HIP(hipMemcpyAsync(out, d->diag_out(), sizeof(double) * kDiagValues, hipMemcpyDeviceToHost,
                        d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  return PF_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char* pf_last_error(void) { return g_last_error.c_str(); }

pf_status pf_set_variant(int32_t variant) {
  if (variant != 0 && variant != 1) return fail(PF_ERR_INVALID_ARG, "variant must be 0 or 1");
  g_variant.store(variant);
  return PF_OK;
}

pf_status pf_required_bytes(const pf_domain_desc* desc, size_t* out) {
  if (!desc || !out) return fail(PF_ERR_INVALID_ARG, "null argument");
  Layout L;
  if (!make_layout(*desc, L)) return fail(PF_ERR_INVALID_ARG, "invalid domain description");
  *out = L.total;
  return PF_OK;
}

pf_status pf_create_domain(const pf_domain_desc* desc, const pf_device_buffer* borrowed,
                           void* stream, pf_domain** out) {
  if (!desc || !out) return fail(PF_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  Layout L;
  if (!make_layout(*desc, L)) return fail(PF_ERR_INVALID_ARG, "invalid domain description");
  pf_domain* d = new (std::nothrow) pf_domain();
  if (!d) return fail(PF_ERR_OOM, "host allocation failed");
  d->desc = *desc;
  d->L = L;
  d->T = choose_tiling(desc->nx, desc->ny, desc->nz, desc->prec);
  d->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&d->device) != hipSuccess) {
    delete d;
    return fail(PF_ERR_DEVICE, "hipGetDevice failed");
  }
  if (borrowed) {
    if (!borrowed->base || borrowed->bytes < L.total ||
        reinterpret_cast<uintptr_t>(borrowed->base) % kAlign != 0) {
      delete d;
      return fail(PF_ERR_INVALID_ARG, "borrowed buffer too small or misaligned");
    }
    d->base = static_cast<char*>(borrowed->base);
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, L.total) != hipSuccess || !p) {
      (void)hipGetLastError();
      delete d;
      return fail(PF_ERR_OOM, "hipMalloc of " + std::to_string(L.total) + " bytes failed");
    }
    d->base = static_cast<char*>(p);
    d->owned = true;
  }
  d->dev = reinterpret_cast<DevDomain*>(d->base + L.off_desc);
  d->dev_ptrs = reinterpret_cast<DevDomain**>(d->base + L.off_ptrs);
  d->dev_first = reinterpret_cast<int32_t*>(d->base + L.off_first);
  DevDomain& h = d->host;
  std::memset(&h, 0, sizeof(h));
  h.nx = desc->nx;
  h.ny = desc->ny;
  h.nz = desc->nz;
  h.pitch = L.pitch;
  h.plane = L.plane;
  h.fstride = L.fstride;
  h.tx = d->T.tx;
  h.ty = d->T.ty;
  h.zc = d->T.zc;
  h.ntx = d->T.ntx;
  h.nty = d->T.nty;
  h.nzc = d->T.nzc;
  h.xmode = d->T.xmode;
  h.rs = d->T.rs;
  h.prec = desc->prec;
  h.steps_left = -1;
  h.copy[0] = d->fields(0);
  h.copy[1] = d->fields(1);
  h.coef = d->base + L.off_coef;
  h.jfree = d->base + L.off_jfree;
  h.nitems = d->T.blocks();
  h.pflag[0] = d->base + L.off_pflag;
  h.pflag[1] = d->base + L.off_pflag + L.pflag_bytes;
  h.pends[0] = d->base + L.off_pflag + 2 * L.pflag_bytes;
  h.pends[1] = d->base + L.off_pflag + 3 * L.pflag_bytes;
  h.pflag_ok[0] = h.pflag_ok[1] = 0;  // the host mirror never vouches for the flags
  h.dx = desc->dx;
  int32_t first[2] = {0, d->T.blocks()};
  DevDomain* self = d->dev;
  pf_status st = PF_OK;
  if (hipMemcpyAsync(d->dev_ptrs, &self, sizeof(self), hipMemcpyHostToDevice, d->stream) !=
          hipSuccess ||
      hipMemcpyAsync(d->dev_first, first, sizeof(first), hipMemcpyHostToDevice, d->stream) !=
          hipSuccess ||
      hipStreamSynchronize(d->stream) != hipSuccess)
    st = fail(PF_ERR_DEVICE, "descriptor upload failed");
  if (st == PF_OK) st = upload_desc(d);
  for (int i = 0; st == PF_OK && i < 4; ++i)
    if (hipEventCreate(&d->ev[i]) != hipSuccess) st = fail(PF_ERR_DEVICE, "hipEventCreate failed");
  if (st == PF_OK && hipStreamSynchronize(d->stream) != hipSuccess)
    st = fail(PF_ERR_DEVICE, "stream synchronisation failed");
  if (st != PF_OK) {
    pf_destroy(d);
    return st;
  }
  *out = d;
  return PF_OK;
}

pf_status pf_set_params(pf_domain* d, const pf_params* p) {
  if (!d || !p) return fail(PF_ERR_INVALID_ARG, "null argument");
  // a member's descriptor and step budget belong to its pack's captured step
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  if (p->diag_every < 0) return fail(PF_ERR_INVALID_ARG, "diag_every must be >= 0");
  if (p->window_z != 0 && (p->window_z < 1 || p->window_z > d->desc.nz - 2))
    return fail(PF_ERR_INVALID_ARG, "window_z must be 0 or in [1, nz-2]");
  if (p->top_bc != 0 && p->top_bc != 1) return fail(PF_ERR_INVALID_ARG, "top_bc must be 0 or 1");
  if (!std::isfinite(p->mu_fill[0]) || !std::isfinite(p->mu_fill[1]))
    return fail(PF_ERR_INVALID_ARG, "mu_fill must be finite");
  double bound = 0.0;
  pf_status st = validate_and_bound(d, *p, bound);
  if (st != PF_OK) return st;
  double dt = p->dt;
  if (!(dt > 0.0)) dt = 0.25 * bound;
  else if (dt > bound)
    return fail(PF_ERR_UNSTABLE, "dt " + std::to_string(dt) + " above the stability bound " +
                                     std::to_string(bound));
  bool aniso = false;
  for (int a = 0; a < NP; ++a)
    for (int b = a + 1; b < NP; ++b) aniso |= p->aniso_delta[a][b] > 0.0;
  DevDomain& h = d->host;
  h.dt = dt;
  h.eps = p->eps;
  h.TE = p->TE;
  h.T0 = p->T0;
  h.G = p->G;
  h.v = p->v;
  h.zoff = p->zoff;
  h.window_z = p->window_z;
  h.top_bc = p->top_bc;
  h.mu_fill[0] = p->mu_fill[0];
  h.mu_fill[1] = p->mu_fill[1];
  std::memcpy(h.chi0, p->chi0, sizeof(h.chi0));
  std::memcpy(h.chi1, p->chi1, sizeof(h.chi1));
  std::memcpy(h.c0, p->c0, sizeof(h.c0));
  std::memcpy(h.c1, p->c1, sizeof(h.c1));
  std::memcpy(h.w0, p->w0, sizeof(h.w0));
  std::memcpy(h.w1, p->w1, sizeof(h.w1));
  std::memcpy(h.D, p->D, sizeof(h.D));
  fill_kparams(h.kp64, *p, dt, d->desc.dx, aniso);
  fill_kparams(h.kp32, *p, dt, d->desc.dx, aniso);
  // keep the device's dynamic state (step, parity) when parameters change
  if (d->fields_set) {
    DevDomain cur;
    if ((st = fetch_state(d, cur)) != PF_OK) return st;
    h.step = cur.step;
    h.parity = cur.parity;
    h.shifts = cur.shifts;
  }
  h.steps_left = -1;
  if ((st = upload_desc(d)) != PF_OK) return st;
  if (h.top_bc) PF_HIP(launch_ghost(d->dev, d->desc.prec, d->desc.nx, d->desc.ny, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  d->dt = dt;
  d->bound = bound;
  d->aniso = aniso;
  d->diag_every = p->diag_every;
  d->params_set = true;
  return PF_OK;
}

pf_status pf_get_dt(const pf_domain* d, double* dt, double* bound) {
  if (!d) return fail(PF_ERR_INVALID_ARG, "null domain");
  if (!d->params_set) return fail(PF_ERR_STATE, "pf_set_params has not been called");
  if (dt) *dt = d->dt;
  if (bound) *bound = d->bound;
  return PF_OK;
}

pf_status pf_init_fields(pf_domain* d, const pf_init* in) {
  if (!d || !in) return fail(PF_ERR_INVALID_ARG, "null argument");
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  // arguments first: a refused call leaves the domain as it was
  if (in->kind == PF_INIT_VORONOI) {
    if (in->nseeds < 0 || in->solid_height < 0)
      return fail(PF_ERR_INVALID_ARG, "nseeds and solid_height must be >= 0");
  } else if (in->kind == PF_INIT_HOST) {
    if (!in->phi || !in->mu) return fail(PF_ERR_INVALID_ARG, "HOST init needs phi and mu");
  } else {
    return fail(PF_ERR_INVALID_ARG, "unknown init kind");
  }
  const pf_domain_desc& g = d->desc;
  const Layout& L = d->L;
  pf_status st;
  // the state lives in copy 0 from now on
  DevDomain& h = d->host;
  if (d->params_set) {
    DevDomain cur;
    if ((st = fetch_state(d, cur)) != PF_OK) return st;
  }
  // until the new fields are complete the domain holds no usable state (a
  // failed call leaves it so: stepping or reading it is refused)
  d->fields_set = false;
  h.step = 0;
  h.parity = 0;
  h.shifts = 0;
  h.shift_now = 0;
  h.steps_left = -1;
  if ((st = upload_desc(d)) != PF_OK) return st;
  // no step has classified the items yet
  PF_HIP(hipMemsetAsync(d->base + d->L.off_jfree + sizeof(uint32_t) * (size_t)count_base(d->T.blocks()),
                        0, sizeof(uint32_t) * kCountWords, d->stream));
  if (in->kind == PF_INIT_VORONOI) {
    std::vector<int8_t> map;
    voronoi_columns(g.nx, g.ny, in->seed, in->nseeds, map);
    int8_t* dmap = reinterpret_cast<int8_t*>(d->base + L.off_map);
    PF_HIP(hipMemcpyAsync(dmap, map.data(), map.size(), hipMemcpyHostToDevice, d->stream));
    PF_HIP(launch_fill(d->dev, g.prec, g.nx, g.ny, g.nz, dmap, in->solid_height, in->mu_init[0],
                       in->mu_init[1], d->stream));
    PF_HIP(hipStreamSynchronize(d->stream));
  } else {  // PF_INIT_HOST
    // each field goes to copy 1 as dense FP64 (a copy holds at least
    // 8 bytes per cell and field: six fields of at least 4 bytes), and a
    // kernel rounds it into copy 0; padding and the ghost planes of copy 0
    // start at zero
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    double* stage = reinterpret_cast<double*>(d->fields(1));
    PF_HIP(hipMemsetAsync(d->fields(0), 0, L.copy_bytes, d->stream));
    for (int f = 0; f < NFIELD; ++f) {
      const double* srcf = f < NP ? in->phi + (size_t)f * n : in->mu + (size_t)(f - NP) * n;
      PF_HIP(hipMemcpyAsync(stage, srcf, sizeof(double) * (size_t)n, hipMemcpyHostToDevice,
                            d->stream));
      PF_HIP(launch_field_unpack(d->dev, g.prec, n, 0, f, stage, d->stream));
    }
    PF_HIP(hipStreamSynchronize(d->stream));
  }
  if (h.top_bc) {
    PF_HIP(launch_ghost(d->dev, g.prec, g.nx, g.ny, d->stream));
    PF_HIP(hipStreamSynchronize(d->stream));
  }
  d->fields_set = true;
  d->since_diag = 0;
  d->diag_pending = false;
  return PF_OK;
}

pf_status pf_set_time(pf_domain* d, int64_t step) {
  pf_status st = check_state(d);
  if (st != PF_OK) return st;
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  if (step < 0) return fail(PF_ERR_INVALID_ARG, "step must be >= 0");
  DevDomain cur;
  if ((st = fetch_state(d, cur)) != PF_OK) return st;
  d->host.step = step;
  d->host.parity = cur.parity;
  d->host.shifts = cur.shifts;
  d->host.steps_left = -1;
  if ((st = upload_desc(d)) != PF_OK) return st;
  PF_HIP(hipStreamSynchronize(d->stream));
  return PF_OK;
}

pf_status pf_step(pf_domain* d, int64_t n) {
  pf_status st = check_state(d);
  if (st != PF_OK) return st;
  if (n < 0) return fail(PF_ERR_INVALID_ARG, "n must be >= 0");
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  for (int64_t i = 0; i < n; ++i) {
    if ((st = enqueue_step(d, nullptr)) != PF_OK) return st;
    if (d->diag_every > 0 && ++d->since_diag >= d->diag_every) {
      d->since_diag = 0;
      PF_HIP(launch_diag(d->dev, d->desc.prec, d->desc.nx, d->desc.ny, d->desc.nz, -1.0,
                         d->partials(), d->diag_out(), d->stream));
      d->diag_pending = true;
    }
  }
  return PF_OK;
}

pf_status pf_step_timed(pf_domain* d, int64_t n, double* phi_ms, double* mu_ms) {
  pf_status st = check_state(d);
  if (st != PF_OK) return st;
  if (n < 0) return fail(PF_ERR_INVALID_ARG, "n must be >= 0");
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  // three events per step, all read after the last step, so the steps run
  // back to back exactly as in pf_step.  They only time: without the
  // system-scope fence an event costs no cache writeback (with it, each
  // added about 5.6 us between the kernels it separates); the stream is
  // synchronised before returning, so the results are visible as after
  // pf_step and pf_sync.
  while (d->timing_events.size() < (size_t)(3 * n)) {
    hipEvent_t e;
    PF_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    d->timing_events.push_back(e);
  }
  for (int64_t i = 0; i < n; ++i)
    if ((st = enqueue_step(d, d->timing_events.data() + 3 * i)) != PF_OK) return st;
  double tp = 0.0, tm = 0.0;
  if (n > 0) PF_HIP(hipEventSynchronize(d->timing_events[3 * n - 1]));
  PF_HIP(hipStreamSynchronize(d->stream));
  for (int64_t i = 0; i < n; ++i) {
    float a = 0.f, b = 0.f;
    hipEvent_t* e = d->timing_events.data() + 3 * i;
    PF_HIP(hipEventElapsedTime(&a, e[0], e[1]));
    PF_HIP(hipEventElapsedTime(&b, e[1], e[2]));
    tp += a;
    tm += b;
  }
  if (phi_ms) *phi_ms += tp;
  if (mu_ms) *mu_ms += tm;
  return PF_OK;
}

pf_status pf_sync(pf_domain* d) {
  if (!d) return fail(PF_ERR_INVALID_ARG, "null domain");
  pf_status sst = sync_domain(d);
  if (sst != PF_OK) return sst;
  if (d->diag_pending) {
    double v[kDiagValues];
    PF_HIP(hipMemcpy(v, d->diag_out(), sizeof(v), hipMemcpyDeviceToHost));
    d->diag_pending = false;
    if (v[9] > 0.0)
      return fail(PF_ERR_NONFINITE, "diagnostics found " + std::to_string((int64_t)v[9]) +
                                        " non-finite cells");
  }
  return PF_OK;
}

pf_status pf_get_step(const pf_domain* d, int64_t* step) {
  if (!d || !step) return fail(PF_ERR_INVALID_ARG, "null argument");
  DevDomain cur;
  pf_status st = fetch_state(const_cast<pf_domain*>(d), cur);
  if (st != PF_OK) return st;
  *step = cur.step;
  return PF_OK;
}

pf_status pf_read_fields(pf_domain* d, double* phi, double* mu, pf_diag* diag) {
  pf_status st = check_state(d);
  if (st != PF_OK) return st;
  DevDomain cur;
  if ((st = fetch_state(d, cur)) != PF_OK) return st;
  const pf_domain_desc& g = d->desc;
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  if (phi || mu) {
    // each field as dense FP64, staged in the copy that does not hold the
    // state (at least 8 bytes per cell and field), then to the host.  That
    // copy will no longer hold the chunks the bulk shortcut may take for
    // equal in both copies: first clear that mark from the current copy's
    // flags (they still describe the current copy, which is unchanged)
    PF_HIP(launch_drop_same(reinterpret_cast<uint8_t*>(d->base + d->L.off_pflag +
                                                       cur.parity * d->L.pflag_bytes),
                            (int64_t)d->L.pflag_bytes, d->stream));
    double* stage = reinterpret_cast<double*>(d->fields(cur.parity ^ 1));
    hipError_t e = hipSuccess;
    for (int f = 0; f < NFIELD && e == hipSuccess; ++f) {
      double* dstf = f < NP ? (phi ? phi + (size_t)f * n : nullptr)
                            : (mu ? mu + (size_t)(f - NP) * n : nullptr);
      if (!dstf) continue;
      e = launch_field_pack(d->dev, g.prec, n, cur.parity, f, stage, d->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dstf, stage, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost,
                           d->stream);
    }
    // the staging covered the ghost planes of that copy: restore them,
    // whatever the outcome of the copies
    if (d->host.top_bc) {
      const hipError_t eg = launch_ghost(d->dev, g.prec, g.nx, g.ny, d->stream);
      if (e == hipSuccess) e = eg;
    }
    const hipError_t es = hipStreamSynchronize(d->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess)
      return fail(PF_ERR_DEVICE, std::string("reading the fields: ") + hipGetErrorString(e));
  }
  if (diag) {
    const double t = (double)cur.step * d->dt;
    double v[kDiagValues];
    if ((st = run_diag(d, t, v)) != PF_OK) return st;
    diag->t = t;
    diag->step = cur.step;
    diag->sum_c[0] = v[0];
    diag->sum_c[1] = v[1];
    for (int a = 0; a < NP; ++a) diag->sum_phi[a] = v[2 + a];
    diag->max_simplex_dev = v[6];
    diag->phi_min = v[7];
    diag->phi_max = v[8];
    diag->nonfinite = (int64_t)v[9];
    diag->window_shifts = cur.shifts;
    uint32_t words[kCountWords];
    PF_HIP(hipMemcpy(words, d->base + d->L.off_jfree + sizeof(uint32_t) * (size_t)count_base(d->T.blocks()),
                     sizeof(words), hipMemcpyDeviceToHost));
    uint32_t counts[kCountKinds] = {};
    for (int k = 0; k < kCountKinds; ++k)
      for (int sl = 0; sl < kCountSlots; ++sl) counts[k] += words[count_word(k, sl)];
    diag->light_items = (int32_t)counts[kCountLight];
    diag->fixed_items = (int32_t)counts[kCountFixed];
    diag->mu_pure_items = (int32_t)counts[kCountPure];
    diag->copied_items = (int32_t)counts[kCountCopied];
    diag->reserved = 0;
    diag->work_items = d->T.ntx * d->T.nty * d->T.nzc;  // without the launch's padding blocks
    if (diag->nonfinite > 0)
      return fail(PF_ERR_NONFINITE, std::to_string(diag->nonfinite) + " non-finite cells");
  }
  return PF_OK;
}

void pf_destroy(pf_domain* d) {
  if (!d) return;
  if (d->pack) (void)pf_pack_remove(d->pack, d);  // never leave a dangling member
  (void)hipStreamSynchronize(d->stream);
  for (auto& e : d->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : d->timing_events) (void)hipEventDestroy(e);
  if (d->owned && d->base) (void)hipFree(d->base);
  delete d;
}

// ---------------------------------------------------------- output path

namespace {

struct CkptHeader {
  char magic[8];
  int32_t nx, ny, nz, prec;
  int64_t step, shifts;
  double dx, dt;
  int64_t zero;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");
constexpr char kCkptMagic[8] = {'P', 'F', 'C', 'K', 'P', 'T', '0', '1'};
constexpr size_t kCkptChunk = (size_t)64 << 20;  // host staging per transfer

struct FileCloser {
  FILE* f;
  ~FileCloser() {
    if (f) std::fclose(f);
  }
};

}  // namespace

pf_status pf_checkpoint_save(pf_domain* d, const char* path) {
  if (!d || !path) return fail(PF_ERR_INVALID_ARG, "null argument");
  if (!d->fields_set) return fail(PF_ERR_STATE, "pf_init_fields has not been called");
  pf_status st;
  DevDomain cur;
  if ((st = fetch_state(d, cur)) != PF_OK) return st;
  const pf_domain_desc& g = d->desc;
  const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
  FileCloser fc{std::fopen(path, "wb")};
  if (!fc.f) return fail(PF_ERR_IO, std::string("cannot open ") + path + " for writing");
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.nx = g.nx;
  h.ny = g.ny;
  h.nz = g.nz;
  h.prec = g.prec;
  h.step = cur.step;
  h.shifts = cur.shifts;
  h.dx = g.dx;
  h.dt = d->dt;
  // stage the rounded fields in the copy that does not hold the state
  float* stage = reinterpret_cast<float*>(d->fields(cur.parity ^ 1));
  PF_HIP(launch_ckpt_pack(d->dev, g.prec, cells, cur.parity, stage, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  const auto write_all = [&]() -> pf_status {
    if (std::fwrite(&h, sizeof(h), 1, fc.f) != 1) return fail(PF_ERR_IO, "checkpoint write failed");
    const size_t total = sizeof(float) * NFIELD * (size_t)cells;
    std::vector<char> buf(std::min(total, kCkptChunk));
    for (size_t o = 0; o < total; o += buf.size()) {
      const size_t n = std::min(buf.size(), total - o);
      PF_HIP(hipMemcpy(buf.data(), reinterpret_cast<char*>(stage) + o, n, hipMemcpyDeviceToHost));
      if (std::fwrite(buf.data(), 1, n, fc.f) != n) return fail(PF_ERR_IO, "checkpoint write failed");
    }
    const int rc = std::fclose(fc.f);
    fc.f = nullptr;
    return rc == 0 ? PF_OK : fail(PF_ERR_IO, "checkpoint write failed");
  };
  st = write_all();
  // the staging block covered the ghost planes of that copy: restore them
  // whatever the outcome of the write; the copy no longer holds the chunks
  // the bulk shortcut may take for equal in both copies: clear that mark
  if (d->host.top_bc) PF_HIP(launch_ghost(d->dev, g.prec, g.nx, g.ny, d->stream));
  PF_HIP(launch_drop_same(reinterpret_cast<uint8_t*>(d->base + d->L.off_pflag +
                                                     cur.parity * d->L.pflag_bytes),
                          (int64_t)d->L.pflag_bytes, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  return st;
}

pf_status pf_checkpoint_load(pf_domain* d, const char* path) {
  if (!d || !path) return fail(PF_ERR_INVALID_ARG, "null argument");
  if (!d->params_set) return fail(PF_ERR_STATE, "pf_set_params has not been called");
  if (d->pack) return fail(PF_ERR_STATE, "domain is a pack member");
  const pf_domain_desc& g = d->desc;
  FileCloser fc{std::fopen(path, "rb")};
  if (!fc.f) return fail(PF_ERR_IO, std::string("cannot open ") + path);
  CkptHeader h{};
  if (std::fread(&h, sizeof(h), 1, fc.f) != 1) return fail(PF_ERR_IO, "checkpoint header short");
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0)
    return fail(PF_ERR_INVALID_ARG, "not a checkpoint file");
  if (h.nx != g.nx || h.ny != g.ny || h.nz != g.nz)
    return fail(PF_ERR_INVALID_ARG, "checkpoint size differs from the domain");
  if (h.step < 0) return fail(PF_ERR_INVALID_ARG, "checkpoint step is negative");
  const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
  // a truncated file is refused before any field is touched
  if (std::fseek(fc.f, 0, SEEK_END) != 0 || std::ftell(fc.f) != (long)(sizeof(CkptHeader) +
                                                                      sizeof(float) * NFIELD * cells) ||
      std::fseek(fc.f, (long)sizeof(CkptHeader), SEEK_SET) != 0)
    return fail(PF_ERR_IO, "checkpoint file has the wrong length");
  pf_status st;
  DevDomain cur;
  if ((st = fetch_state(d, cur)) != PF_OK) return st;
  // read into copy 1, widen into copy 0, which then holds the state; from
  // the first write on, the old state may be gone: until the load has
  // completed the domain holds no usable state (a failed load leaves it so)
  d->fields_set = false;
  float* stage = reinterpret_cast<float*>(d->fields(1));
  const size_t total = sizeof(float) * NFIELD * (size_t)cells;
  std::vector<char> buf(std::min(total, kCkptChunk));
  for (size_t o = 0; o < total; o += buf.size()) {
    const size_t n = std::min(buf.size(), total - o);
    if (std::fread(buf.data(), 1, n, fc.f) != n) return fail(PF_ERR_IO, "checkpoint data short");
    PF_HIP(hipMemcpy(reinterpret_cast<char*>(stage) + o, buf.data(), n, hipMemcpyHostToDevice));
  }
  DevDomain& hd = d->host;
  hd.step = h.step;
  hd.parity = 0;
  hd.shifts = h.shifts;
  hd.shift_now = 0;
  hd.steps_left = -1;
  if ((st = upload_desc(d)) != PF_OK) return st;
  PF_HIP(hipMemsetAsync(d->base + d->L.off_jfree + sizeof(uint32_t) * (size_t)count_base(d->T.blocks()),
                        0, sizeof(uint32_t) * kCountWords, d->stream));
  PF_HIP(launch_ckpt_unpack(d->dev, g.prec, cells, 0, stage, d->stream));
  if (hd.top_bc) PF_HIP(launch_ghost(d->dev, g.prec, g.nx, g.ny, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  d->fields_set = true;
  d->since_diag = 0;
  d->diag_pending = false;
  return PF_OK;
}

pf_status pf_mesh_phase(pf_domain* d, int32_t phase, double iso, const pf_device_buffer* out,
                        int64_t* ntri) {
  if (!d || !out || !ntri) return fail(PF_ERR_INVALID_ARG, "null argument");
  if (phase < 0 || phase >= NP) return fail(PF_ERR_INVALID_ARG, "phase must be 0..3");
  if (!std::isfinite(iso)) return fail(PF_ERR_INVALID_ARG, "iso must be finite");
  if (out->bytes > 0 && (!out->base || reinterpret_cast<uintptr_t>(out->base) % 4 != 0))
    return fail(PF_ERR_INVALID_ARG, "mesh buffer null or misaligned");
  if (!d->fields_set) return fail(PF_ERR_STATE, "pf_init_fields has not been called");
  pf_status st;
  DevDomain cur;
  if ((st = fetch_state(d, cur)) != PF_OK) return st;
  const pf_domain_desc& g = d->desc;
  const int64_t rows = (int64_t)g.ny * (int64_t)(g.nz - 1);  // < 2^31: the layout limits items
  const int64_t cap = (int64_t)(out->bytes / (9 * sizeof(float)));
  auto* count = reinterpret_cast<unsigned long long*>(d->base + d->L.off_mesh);
  PF_HIP(hipMemsetAsync(count, 0, sizeof(*count), d->stream));
  if (rows > 0)
    PF_HIP(launch_mesh(d->dev, g.prec, rows, phase, iso, static_cast<float*>(out->base), cap,
                       count, d->stream));
  unsigned long long n = 0;
  PF_HIP(hipMemcpyAsync(&n, count, sizeof(n), hipMemcpyDeviceToHost, d->stream));
  PF_HIP(hipStreamSynchronize(d->stream));
  *ntri = (int64_t)n;
  if ((int64_t)n > cap)
    return fail(PF_ERR_INVALID_ARG, "mesh needs " + std::to_string(n) + " triangles, buffer holds " +
                                        std::to_string(cap));
  return PF_OK;
}

}  // extern "C"

// ============================================= diagnostics without allocation

// Scratch of pf_diag_fields_noalloc: the partial sums of the diagnostics'
// fixed grid (kDiagBlocks x kDiagValues) and their final values, 38.5 KiB.
// Each device the library runs on holds its own copy until the process
// ends.  Host code never passes this name to a kernel or a copy: it stands
// for the array only on the device side; the per-device address comes from
// hipGetSymbolAddress below.
constexpr size_t kNoAllocDoubles = (size_t)kDiagBlocks * kDiagValues + kDiagValues;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];    // one call at a time per device
double* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

extern "C" {

pf_status pf_diag_fields_noalloc(const pf_domain_desc* desc, const pf_params* p,
                                 const void* fields, double t, void* stream, pf_diag* out) {
  if (!desc || !p || !fields || !out) return fail(PF_ERR_INVALID_ARG, "null argument");
  if (desc->nx <= 0 || desc->ny <= 0 || desc->nz <= 0)
    return fail(PF_ERR_INVALID_ARG, "sizes must be positive");
  if (desc->prec != PF_FP64 && desc->prec != PF_FP32)
    return fail(PF_ERR_INVALID_ARG, "unknown precision");
  if (!(desc->dx > 0.0) || !std::isfinite(desc->dx))
    return fail(PF_ERR_INVALID_ARG, "dx must be positive and finite");
  if (!std::isfinite(t)) return fail(PF_ERR_INVALID_ARG, "t must be finite");
  const size_t elem = desc->prec == PF_FP64 ? 8 : 4;
  const long double bytes = (long double)desc->nx * desc->ny * desc->nz * NFIELD * elem;
  if (bytes > (long double)(1ull << 62))
    return fail(PF_ERR_INVALID_ARG, "fields larger than 2^62 bytes");
  if (reinterpret_cast<uintptr_t>(fields) % elem != 0)
    return fail(PF_ERR_INVALID_ARG, "fields not aligned to their element size");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PF_ERR_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PF_ERR_INVALID_ARG, "device index beyond " + std::to_string(kMaxDevices - 1));
  std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
  if (!g_scratch_ptr[dev]) {  // first call on this device, which is current
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  double* partials = g_scratch_ptr[dev];
  double* final_v = partials + (size_t)kDiagBlocks * kDiagValues;
  DiagView v{};
  v.base = fields;
  v.nx = desc->nx;
  v.ny = desc->ny;
  v.nz = desc->nz;
  v.pitch = desc->nx;
  v.plane = (int64_t)desc->nx * desc->ny;
  v.fstride = v.plane * desc->nz;
  v.T0 = p->T0;
  v.G = p->G;
  v.dx = desc->dx;
  v.zoff = p->zoff;
  v.v = p->v;
  v.TE = p->TE;
  v.shifts = 0;
  std::memcpy(v.chi0, p->chi0, sizeof(v.chi0));
  std::memcpy(v.chi1, p->chi1, sizeof(v.chi1));
  std::memcpy(v.c0, p->c0, sizeof(v.c0));
  std::memcpy(v.c1, p->c1, sizeof(v.c1));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double r[kDiagValues];
  PF_HIP(launch_diag_view(v, desc->prec, t, partials, final_v, s));
  PF_HIP(hipMemcpyAsync(r, final_v, sizeof(r), hipMemcpyDeviceToHost, s));
  PF_HIP(hipStreamSynchronize(s));
  std::memset(out, 0, sizeof(*out));
  out->t = t;
  out->step = -1;
  out->sum_c[0] = r[0];
  out->sum_c[1] = r[1];
  for (int a = 0; a < NP; ++a) out->sum_phi[a] = r[2 + a];
  out->max_simplex_dev = r[6];
  out->phi_min = r[7];
  out->phi_max = r[8];
  out->nonfinite = (int64_t)r[9];
  if (out->nonfinite > 0)
    return fail(PF_ERR_NONFINITE, std::to_string(out->nonfinite) + " non-finite cells");
  return PF_OK;
}

}  // extern "C"

// ==================================================================== packs

struct pf_pack {
  int32_t prec;
  hipStream_t stream;
  int32_t max_domains;
  std::vector<pf_domain*> members;
  DevDomain** dev_ptrs = nullptr;
  int32_t* dev_first = nullptr;
  int32_t total = 0;
  bool any_aniso = false;
  bool any_window = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;
  bool own_stream = false;  // created here because the caller passed NULL
};

namespace {

void drop_graph(pf_pack* pk) {
  if (pk->exec) (void)hipGraphExecDestroy(pk->exec);
  if (pk->graph) (void)hipGraphDestroy(pk->graph);
  pk->exec = nullptr;
  pk->graph = nullptr;
}

pf_status rebuild_pack(pf_pack* pk) {
  std::vector<DevDomain*> ptrs;
  std::vector<int32_t> first(1, 0);
  pk->any_aniso = false;
  pk->any_window = false;
  for (pf_domain* d : pk->members) {
    ptrs.push_back(d->dev);
    first.push_back(first.back() + d->T.blocks());
    pk->any_aniso |= d->aniso;
    pk->any_window |= d->host.window_z > 0;
  }
  pk->total = first.back();
  if (!ptrs.empty()) {
    PF_HIP(hipMemcpyAsync(pk->dev_ptrs, ptrs.data(), sizeof(DevDomain*) * ptrs.size(),
                          hipMemcpyHostToDevice, pk->stream));
    PF_HIP(hipMemcpyAsync(pk->dev_first, first.data(), sizeof(int32_t) * first.size(),
                          hipMemcpyHostToDevice, pk->stream));
    PF_HIP(hipStreamSynchronize(pk->stream));
  }
  drop_graph(pk);
  if (!ptrs.empty()) {
    LaunchSet s;
    s.doms = pk->dev_ptrs;
    s.first = pk->dev_first;
    s.ndom = (int32_t)ptrs.size();
    s.total = pk->total;
    s.words = nullptr;
    const int var = g_variant.load();
    PF_HIP(hipStreamBeginCapture(pk->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = launch_prologue(s, pk->prec, pk->stream);
    if (e1 == hipSuccess && pk->any_window) e1 = launch_window(s, pk->prec, pk->stream);
    hipError_t e2 = launch_phi(s, pk->prec, pk->any_aniso, var, pk->stream);
    hipError_t e3 = launch_mu(s, pk->prec, var, pk->stream);
    hipError_t e4 = hipStreamEndCapture(pk->stream, &pk->graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
      return fail(PF_ERR_DEVICE, "pack step capture failed");
    PF_HIP(hipGraphInstantiate(&pk->exec, pk->graph, nullptr, nullptr, 0));
  }
  pk->dirty = false;
  return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_pack_create(int32_t prec, void* stream, int32_t max_domains, pf_pack** out) {
  if (!out) return fail(PF_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (prec != PF_FP64 && prec != PF_FP32) return fail(PF_ERR_INVALID_ARG, "bad precision");
  if (max_domains <= 0 || max_domains > 4096) return fail(PF_ERR_INVALID_ARG, "bad max_domains");
  pf_pack* pk = new (std::nothrow) pf_pack();
  if (!pk) return fail(PF_ERR_OOM, "host allocation failed");
  pk->prec = prec;
  pk->stream = static_cast<hipStream_t>(stream);
  pk->max_domains = max_domains;
  if (!pk->stream) {  // graphs cannot be captured on the null stream
    if (hipStreamCreate(&pk->stream) != hipSuccess) {
      delete pk;
      return fail(PF_ERR_DEVICE, "pack stream creation failed");
    }
    pk->own_stream = true;
  }
  void* p = nullptr;
  const size_t bytes = align_up(sizeof(DevDomain*) * max_domains, kAlign) +
                       sizeof(int32_t) * (max_domains + 1);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (pk->own_stream) (void)hipStreamDestroy(pk->stream);
    delete pk;
    return fail(PF_ERR_OOM, "pack table allocation failed");
  }
  pk->dev_ptrs = static_cast<DevDomain**>(p);
  pk->dev_first = reinterpret_cast<int32_t*>(static_cast<char*>(p) +
                                             align_up(sizeof(DevDomain*) * max_domains, kAlign));
  *out = pk;
  return PF_OK;
}

pf_status pf_pack_add(pf_pack* pk, pf_domain* d, int64_t nsteps) {
  if (!pk || !d) return fail(PF_ERR_INVALID_ARG, "null argument");
  pf_status st = check_state(d);
  if (st != PF_OK) return st;
  if (d->pack) return fail(PF_ERR_STATE, "domain already in a pack");
  if (d->desc.prec != pk->prec) return fail(PF_ERR_INVALID_ARG, "precision mismatch");
  if ((int32_t)pk->members.size() >= pk->max_domains) return fail(PF_ERR_STATE, "pack is full");
  if (nsteps < 0) return fail(PF_ERR_INVALID_ARG, "nsteps must be >= 0");
  PF_HIP(hipStreamSynchronize(d->stream));
  PF_HIP(hipStreamSynchronize(pk->stream));
  PF_HIP(hipMemcpy(reinterpret_cast<char*>(d->dev) + offsetof(DevDomain, steps_left), &nsteps,
                   sizeof(nsteps), hipMemcpyHostToDevice));
  pk->members.push_back(d);
  d->pack = pk;
  d->pack_stream = pk->stream;
  pk->dirty = true;
  return PF_OK;
}

pf_status pf_pack_remove(pf_pack* pk, pf_domain* d) {
  if (!pk || !d) return fail(PF_ERR_INVALID_ARG, "null argument");
  auto it = std::find(pk->members.begin(), pk->members.end(), d);
  if (it == pk->members.end()) return fail(PF_ERR_INVALID_ARG, "not a member");
  PF_HIP(hipStreamSynchronize(pk->stream));
  int64_t unlimited = -1;
  PF_HIP(hipMemcpy(reinterpret_cast<char*>(d->dev) + offsetof(DevDomain, steps_left), &unlimited,
                   sizeof(unlimited), hipMemcpyHostToDevice));
  pk->members.erase(it);
  d->pack = nullptr;
  d->pack_stream = nullptr;
  pk->dirty = true;
  return PF_OK;
}

pf_status pf_pack_remaining(pf_pack* pk, const pf_domain* d, int64_t* left) {
  if (!pk || !d || !left) return fail(PF_ERR_INVALID_ARG, "null argument");
  PF_HIP(hipStreamSynchronize(pk->stream));
  PF_HIP(hipMemcpy(left, reinterpret_cast<const char*>(d->dev) + offsetof(DevDomain, steps_left),
                   sizeof(int64_t), hipMemcpyDeviceToHost));
  return PF_OK;
}

pf_status pf_pack_step(pf_pack* pk, int64_t rounds, int32_t* n_finished) {
  if (!pk) return fail(PF_ERR_INVALID_ARG, "null pack");
  if (rounds < 0) return fail(PF_ERR_INVALID_ARG, "rounds must be >= 0");
  pf_status st;
  if (pk->dirty && (st = rebuild_pack(pk)) != PF_OK) return st;
  if (pk->exec)
    for (int64_t r = 0; r < rounds; ++r) PF_HIP(hipGraphLaunch(pk->exec, pk->stream));
  if (n_finished) {
    PF_HIP(hipStreamSynchronize(pk->stream));
    int32_t fin = 0;
    for (pf_domain* d : pk->members) {
      int64_t left = 0;
      PF_HIP(hipMemcpy(&left, reinterpret_cast<char*>(d->dev) + offsetof(DevDomain, steps_left),
                       sizeof(left), hipMemcpyDeviceToHost));
      fin += left == 0;
    }
    *n_finished = fin;
  }
  return PF_OK;
}

pf_status pf_pack_sync(pf_pack* pk) {
  if (!pk) return fail(PF_ERR_INVALID_ARG, "null pack");
  PF_HIP(hipStreamSynchronize(pk->stream));
  return PF_OK;
}

void pf_pack_destroy(pf_pack* pk) {
  if (!pk) return;
  (void)hipStreamSynchronize(pk->stream);
  for (pf_domain* d : pk->members) {
    d->pack = nullptr;
    d->pack_stream = nullptr;
  }
  drop_graph(pk);
  if (pk->dev_ptrs) (void)hipFree(pk->dev_ptrs);
  if (pk->own_stream) (void)hipStreamDestroy(pk->stream);
  delete pk;
}

}  // extern "C"
