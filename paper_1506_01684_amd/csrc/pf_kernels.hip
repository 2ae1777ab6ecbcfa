// pf_kernels.hip -- HIP kernels of the phase-field time step for gfx950.
//
// One step (Algorithm 1 of the paper) is three stages on one stream:
//   prologue: choice of source/destination copy, step counter, then the
//             per-plane temperature coefficients of the step in FP64
//             (Sec. 3.3);
//   phi-sweep: phi_dst <- (phi_src, mu_src)             (Eqs. (1)-(2));
//   mu-sweep:  mu_dst  <- (mu_src, phi_src, phi_dst)     (Eqs. (3)-(4)).
// Boundaries are applied by index arithmetic (periodic x/y, mirror z), so
// there are no ghost layers and no separate boundary pass.
//
// This file holds the prologue, the "direct" variant of both sweeps (one
// thread per cell evaluating all six faces), the Voronoi fill and the
// diagnostics reduction.  The face-sharing z-marching variant is in
// pf_tiled.hip.
#include <hip/hip_runtime.h>

#include "pf_device.h"
#include "pf_kernels_common.h"
#include "pf_launch.h"

namespace pfk {

// ------------------------------------------------------------- prologue

// One work group per domain.  Records the source copy of step n = d.step
// (after a moving-window shift, if the front has passed the window plane),
// zeroes the step's item counts, marks the first plane of every z chunk for
// the fixed-point reduction of coef_kernel, then advances the step counter
// and the parity.  A domain whose step budget is spent is marked inactive
// and left untouched.
template <typename R>
__global__ __launch_bounds__(256) void prologue_kernel(DevDomain* const* doms, int ndom) {
  DevDomain& d = *doms[blockIdx.x];
  __shared__ int64_t s_step;
  __shared__ int s_src, s_act;
  __shared__ double s_red[256];
  if (threadIdx.x == 0) {
    int act = d.steps_left != 0;
    s_act = act;
    s_step = d.step;
    s_src = d.parity;
  }
  __syncthreads();
  if (!s_act) {
    if (threadIdx.x == 0) d.active = 0;
    return;
  }
  // counts of this step's items that the phi-sweep finds free of
  // anti-trapping faces, that it copies unchanged, and that the mu-sweep
  // evaluates from mu alone
  if (threadIdx.x < kCountKinds * kCountSlots)
    static_cast<uint32_t*>(d.jfree)[count_base(d.nitems) +
                                    count_word(threadIdx.x / kCountSlots, threadIdx.x % kCountSlots)] = 0u;
  // Moving window: has the front passed plane window_z?  The liquid
  // fraction of that plane of the current state is summed in FP64 (strided
  // per thread, then a fixed tree); below half the plane area the step
  // starts with a shift, which the window kernel performs by copying the
  // current copy into the other one, one plane lower.
  int shift = 0;
  if (d.window_z > 0) {
    const R* pl = static_cast<const R*>(d.copy[s_src]) + 3 * d.fstride + (int64_t)d.window_z * d.plane;
    double acc = 0.0;
    // rows of the plane over the threads, eight loads in flight per thread
    const int n = d.nx * d.ny;
    int c = threadIdx.x;
    for (; c + 7 * (int)blockDim.x < n; c += 8 * blockDim.x) {
      R v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int cu = c + u * blockDim.x;
        v[u] = pl[(int64_t)(cu / d.nx) * d.pitch + cu % d.nx];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; c < n; c += blockDim.x) acc += (double)pl[(int64_t)(c / d.nx) * d.pitch + c % d.nx];
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
      __syncthreads();
    }
    shift = s_red[0] < 0.5 * (double)d.nx * (double)d.ny;
  }
  const int src = shift ? s_src ^ 1 : s_src;
  const int64_t n = s_step;
  // each chunk's fixed-point mask starts full; coef_kernel ANDs every plane in
  PlaneCoef<R>* tab = static_cast<PlaneCoef<R>*>(d.coef);
  for (int iz = threadIdx.x; iz < d.nzc; iz += blockDim.x) tab[iz * d.zc].chunk_fixed = ~0;
  __syncthreads();
  if (threadIdx.x == 0) {
    // the pure-phase flags of the copy this step writes are renewed by the
    // tiled phi-sweep; a shifted state invalidates those of its copy
    d.pflag_ok[src ^ 1] = 0;
    if (shift) d.pflag_ok[src] = 0;
    d.active = 1;
    d.cur_step = n;
    d.shift_now = shift;
    d.shift_src = s_src;
    d.shifts += shift;
    d.cur_src = src;
    d.step = n + 1;
    d.parity = src ^ 1;
    if (d.steps_left > 0) d.steps_left -= 1;
  }
}

// Per-plane coefficients of the running step n = d.cur_step at
// t_n = n dt and t_{n+1} = (n+1) dt (products, never sums), evaluated in
// FP64 and rounded to R (Sec. 3.3: everything that depends only on the
// temperature once per z slice).  kCoefBlocks work groups per domain; four
// threads per plane, thread a of a plane also evaluating what depends on
// phase a (the pure-item coefficients and the fixed-point test), so that
// the planes' longest chain is one phase's cell stage rather than four.
// Each plane ANDs its fixed-point mask into its chunk's first record.
template <typename R>
__global__ __launch_bounds__(kCoefThreads) void coef_kernel(DevDomain* const* doms, int ndom) {
  const DevDomain& d = *doms[blockIdx.x / kCoefBlocks];
  if (!d.active) return;
  const int a = threadIdx.x & 3;
  const double zoff = d.zoff + (double)d.shifts * d.dx;
  const int64_t n = d.cur_step;
  const double t0 = (double)n * d.dt, t1 = (double)(n + 1) * d.dt;
  PlaneCoef<R>* tab = static_cast<PlaneCoef<R>*>(d.coef);
  for (int k0 = (blockIdx.x % kCoefBlocks) * (kCoefThreads / 4); k0 < d.nz;
       k0 += kCoefBlocks * (kCoefThreads / 4)) {
    const int k = k0 + (int)(threadIdx.x >> 2);
    // every lane takes part in the shuffles below; lanes past the last
    // plane evaluate plane nz-1 and write nothing
    const int kc = k < d.nz ? k : d.nz - 1;
    const double zc = (double)kc * d.dx + zoff;
    const double Tn = d.T0 + d.G * (zc - d.v * t0);
    const double Tz = d.T0 + d.G * (zc + 0.5 * d.dx - d.v * t0);
    const double Tn1 = d.T0 + d.G * (zc - d.v * t1);
    PlaneCoef<R> c;
    c.epsT = (R)(d.eps * Tn);
    c.Toe = (R)(Tn / d.eps);
    double chiN[NP][NM], cbN[NP][NM], chiZ[NP][NM], cbZ[NP][NM];
    for (int b = 0; b < NP; ++b) {
      c.wbar[b] = (R)(d.w0[b] + d.w1[b] * (Tn - d.TE));
      for (int q = 0; q < NM; ++q) {
        chiN[b][q] = d.chi0[b][q] + d.chi1[b][q] * (Tn - d.TE);
        cbN[b][q] = d.c0[b][q] + d.c1[b][q] * (Tn - d.TE);
        chiZ[b][q] = d.chi0[b][q] + d.chi1[b][q] * (Tz - d.TE);
        cbZ[b][q] = d.c0[b][q] + d.c1[b][q] * (Tz - d.TE);
        const double chiN1 = d.chi0[b][q] + d.chi1[b][q] * (Tn1 - d.TE);
        const double cbN1 = d.c0[b][q] + d.c1[b][q] * (Tn1 - d.TE);
        c.chi[b][q] = (R)chiN[b][q];
        c.cbar[b][q] = (R)cbN[b][q];
        c.Dchi[b][q] = (R)(d.D[b] * chiN[b][q]);
        c.DchiZ[b][q] = (R)(d.D[b] * chiZ[b][q]);
        c.chi1[b][q] = (R)chiN1;
        c.dchi[b][q] = (R)(chiN1 - chiN[b][q]);
        c.dcbar[b][q] = (R)(cbN1 - cbN[b][q]);
      }
    }
    for (int b = 0; b < 3; ++b)
      for (int q = 0; q < NM; ++q) {
        c.dchiL[b][q] = (R)(chiN[LQ][q] - chiN[b][q]);
        c.dcbL[b][q] = (R)(cbN[LQ][q] - cbN[b][q]);
        c.dchiLZ[b][q] = (R)(chiZ[LQ][q] - chiZ[b][q]);
        c.dcbLZ[b][q] = (R)(cbZ[LQ][q] - cbZ[b][q]);
      }
    // coefficients of the mu-sweep of pure-a items (mu_pure_item)
    R e[NP], h[NP], Mp[NM], MpZ[NM], rchip[NM];
    for (int b = 0; b < NP; ++b) e[b] = b == a ? R(1) : R(0);
    mu_cell_h<R>(e, h);
    mu_face_m<R, false>(c, e, Mp);
    mu_face_m<R, true>(c, e, MpZ);
    for (int q = 0; q < NM; ++q) rchip[q] = rcp_(mu_cell_chi<R>(c, q, h));
    // A pure cell (phi = e_a) whose face terms vanish (A = 0) is a fixed
    // point when the cell stage maps it to e_a exactly.  Decided by running
    // that cell stage (phi_cell in the path's precision) on e_a with A = 0:
    // its driving force is zero for every finite mu (h = e_a, so
    // psi_a - sum h psi = 0 and phi_b = 0 multiplies the rest), so mu = 0
    // stands for any state.  As a guard against a different fusion of the
    // same arithmetic where the sweep inlines it, the step must also keep
    // a clear margin: rhs_a = 0, rhs_b = (T/eps) 16/pi^2 gamma_ab, so
    // y_a = 1 + rate_a m and y_b = -rate_b (rhs_b - m) (m the mean), and
    // the projection returns e_a when every y_b stays below y_a - 1; the
    // margin is relative, plus an absolute 2^-20 for the rounding of y_a
    // near 1 in FP32.
    bool fixed;
    {
      R A[NP], m0[NM] = {R(0), R(0)};
      for (int b = 0; b < NP; ++b) A[b] = R(0);
      double out[NP];
      phi_cell<R>(kparams<R>(d), c, e, m0, A, out);
      fixed = true;
      for (int b = 0; b < NP; ++b) fixed = fixed && (R)out[b] == e[b];
      double rhs[NP], m = 0.0;
      for (int b = 0; b < NP; ++b) {
        rhs[b] = b == a ? 0.0 : (Tn / d.eps) * d.kp64.g16[a < b ? pair_index(a, b) : pair_index(b, a)];
        m += rhs[b];
      }
      m *= 0.25;
      const double thr = d.kp64.rate[a] * m;
      for (int b = 0; b < NP; ++b) {
        if (b == a) continue;
        const double yb = -d.kp64.rate[b] * (rhs[b] - m);
        fixed = fixed && yb + 1e-5 * (fabs(thr) + fabs(yb)) + 0x1p-20 < thr;
      }
    }
    // the four phases' bits of the plane (lanes 4j .. 4j+3 of the wave)
    int bits = fixed ? 1 << a : 0;
    bits |= __shfl_xor(bits, 1);
    bits |= __shfl_xor(bits, 2);
    if (k >= d.nz) continue;
    PlaneCoef<R>& o = tab[k];
    for (int q = 0; q < NM; ++q) {
      o.Mp[a][q] = Mp[q];
      o.MpZ[a][q] = MpZ[q];
      o.rchip[a][q] = rchip[q];
    }
    if (a != 0) continue;
    o.epsT = c.epsT;
    o.Toe = c.Toe;
    for (int b = 0; b < NP; ++b) {
      o.wbar[b] = c.wbar[b];
      for (int q = 0; q < NM; ++q) {
        o.chi[b][q] = c.chi[b][q];
        o.cbar[b][q] = c.cbar[b][q];
        o.Dchi[b][q] = c.Dchi[b][q];
        o.DchiZ[b][q] = c.DchiZ[b][q];
        o.chi1[b][q] = c.chi1[b][q];
        o.dchi[b][q] = c.dchi[b][q];
        o.dcbar[b][q] = c.dcbar[b][q];
      }
    }
    for (int b = 0; b < 3; ++b)
      for (int q = 0; q < NM; ++q) {
        o.dchiL[b][q] = c.dchiL[b][q];
        o.dcbL[b][q] = c.dcbL[b][q];
        o.dchiLZ[b][q] = c.dchiLZ[b][q];
        o.dcbLZ[b][q] = c.dcbLZ[b][q];
      }
    o.pure_fixed = bits;
    // the fixed points of every plane of each z chunk, at its first plane
    // (set to all ones by the prologue; other planes keep all ones)
    if (k % d.zc != 0) o.chunk_fixed = ~0;
    atomicAnd(&tab[k / d.zc * d.zc].chunk_fixed, bits);
  }
}

// Window shift of the domains whose prologue decided one: the running
// source copy (cur_src) receives the state of copy shift_src moved down by
// one plane, with a liquid plane at mu_fill on top.  Work items are the
// sweeps' (tile, z chunk) items; each thread copies its column.
template <typename R>
__global__ __launch_bounds__(kTileThreads) void window_kernel(DevDomain* const* doms,
                                                              const int32_t* first, int ndom,
                                                              int total) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int di = find_domain(first, ndom, item);
    const PF_CONST DevDomain& d = domain_at(doms, di);
    if (!d.active || !d.shift_now) continue;
    const WorkTile w = decode_item(d, item - first_item(first, di), threadIdx.x);
    if (!w.valid) continue;
    const R* from = static_cast<const R*>(d.copy[d.shift_src]);
    R* to = static_cast<R*>(d.copy[d.cur_src]);
    const int64_t col = (int64_t)w.y * d.pitch + w.x;
    for (int k = w.z0; k < w.z1; ++k) {
      const bool top = k == d.nz - 1;
      const int64_t o = (int64_t)k * d.plane + col;
      const int64_t os = (int64_t)(top ? k : k + 1) * d.plane + col;  // never past plane nz-1
#pragma unroll
      for (int f = 0; f < NP + NM; ++f) {
        const R fill = f < NP ? (f == LQ ? R(1) : R(0)) : (R)d.mu_fill[f - NP];
        const R v = from[f * d.fstride + os];
        to[f * d.fstride + o] = top ? fill : v;
      }
    }
  }
}

// ------------------------------------------------------- direct variant

// Gather the face inputs of the face between L=(xl,yl,zl) and U (normal D):
// face averages pb, normal differences gn and, when FULL, the tangential
// components gt1, gt2 (axes in increasing order, skipping D), each the
// average of the central differences at L and U (4-point stencil).
template <typename R, int D, bool FULL>
__device__ __forceinline__ void gather_face(const PF_GLOBAL R* const* f, const Geo& g, int xl,
                                            int yl, int zl, R inv_dx, R inv_4dx, R pb[NP],
                                            R gn[NP], R gt1[NP], R gt2[NP]) {
  const int xu = D == 0 ? g.xp(xl) : xl;
  const int yu = D == 1 ? g.yp(yl) : yl;
  const int zu = D == 2 ? zl + 1 : zl;
  const int64_t oL = g.at(xl, yl, zl), oU = g.at(xu, yu, zu);
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    const R uL = f[a][oL], uU = f[a][oU];
    pb[a] = R(0.5) * (uL + uU);
    gn[a] = (uU - uL) * inv_dx;
    gt1[a] = gt2[a] = R(0);
  }
  if constexpr (FULL) {
    constexpr int t1 = D == 0 ? 1 : 0;
    constexpr int t2 = D == 2 ? 1 : 2;
    int64_t o1[4], o2[4];  // L+, U+, L-, U-
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int tt = s == 0 ? t1 : t2;
      int64_t* o = s == 0 ? o1 : o2;
      if (tt == 0) {
        o[0] = g.at(g.xp(xl), yl, zl); o[1] = g.at(g.xp(xu), yu, zu);
        o[2] = g.at(g.xm(xl), yl, zl); o[3] = g.at(g.xm(xu), yu, zu);
      } else if (tt == 1) {
        o[0] = g.at(xl, g.yp(yl), zl); o[1] = g.at(xu, g.yp(yu), zu);
        o[2] = g.at(xl, g.ym(yl), zl); o[3] = g.at(xu, g.ym(yu), zu);
      } else {
        o[0] = g.at(xl, yl, g.zp(zl)); o[1] = g.at(xu, yu, g.zp(zu));
        o[2] = g.at(xl, yl, g.zm(zl)); o[3] = g.at(xu, yu, g.zm(zu));
      }
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      gt1[a] = ((f[a][o1[0]] + f[a][o1[1]]) - (f[a][o1[2]] + f[a][o1[3]])) * inv_4dx;
      gt2[a] = ((f[a][o2[0]] + f[a][o2[1]]) - (f[a][o2[2]] + f[a][o2[3]])) * inv_4dx;
    }
  }
}

template <typename R, bool ANISO, int D, typename KP>
__device__ __forceinline__ void phi_face_at(const KP& P, const PF_GLOBAL R* const* f,
                                            const Geo& g, int xl, int yl, int zl, R F[NP],
                                            R S[NP]) {
  if (D == 2 && !g.zface(zl)) {  // zero-flux z boundary
#pragma unroll
    for (int a = 0; a < NP; ++a) F[a] = S[a] = R(0);
    return;
  }
  R pb[NP], gn[NP], gt1[NP], gt2[NP];
  gather_face<R, D, ANISO>(f, g, xl, yl, zl, (R)P.inv_dx, (R)P.inv_4dx, pb, gn, gt1, gt2);
  phi_face<R, ANISO, D>(P, pb, gn, gt1, gt2, F, S);
}

template <typename R, bool ANISO>
__global__ __launch_bounds__(kTileThreads) void phi_direct_kernel(DevDomain* const* doms,
                                                                  const int32_t* first, int ndom,
                                                                  int total) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int di = find_domain(first, ndom, item);
    const PF_CONST DevDomain& d = domain_at(doms, di);
    if (!d.active) continue;
    const WorkTile w = decode_item(d, item - first_item(first, di), threadIdx.x);
    if (!w.valid) continue;
    const Geo g = make_geo(d);
    const auto& P = kparams<R>(d);
    const PF_CONST PlaneCoef<R>* tab = to_const(static_cast<const PlaneCoef<R>*>(d.coef));
    const PF_GLOBAL R* src = to_global(static_cast<const R*>(d.copy[d.cur_src]));
    PF_GLOBAL R* dst = to_global(static_cast<R*>(d.copy[d.cur_src ^ 1]));
    const int64_t fs = d.fstride;
    const PF_GLOBAL R* ph[NP] = {src, src + fs, src + 2 * fs, src + 3 * fs};
    const PF_GLOBAL R* mu[NM] = {src + 4 * fs, src + 5 * fs};
    const int x = w.x, y = w.y;
    const int xm = g.xm(x), ym = g.ym(y);
    for (int k = w.z0; k < w.z1; ++k) {
      R Fu[NP], Su[NP], Fl[NP], Sl[NP], Ss[NP], Fd[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) Ss[a] = Fd[a] = R(0);
      phi_face_at<R, ANISO, 0>(P, ph, g, x, y, k, Fu, Su);
      phi_face_at<R, ANISO, 0>(P, ph, g, xm, y, k, Fl, Sl);
#pragma unroll
      for (int a = 0; a < NP; ++a) { Ss[a] += Su[a] + Sl[a]; Fd[a] += Fu[a] - Fl[a]; }
      phi_face_at<R, ANISO, 1>(P, ph, g, x, y, k, Fu, Su);
      phi_face_at<R, ANISO, 1>(P, ph, g, x, ym, k, Fl, Sl);
#pragma unroll
      for (int a = 0; a < NP; ++a) { Ss[a] += Su[a] + Sl[a]; Fd[a] += Fu[a] - Fl[a]; }
      phi_face_at<R, ANISO, 2>(P, ph, g, x, y, k, Fu, Su);
      phi_face_at<R, ANISO, 2>(P, ph, g, x, y, k - 1, Fl, Sl);
#pragma unroll
      for (int a = 0; a < NP; ++a) { Ss[a] += Su[a] + Sl[a]; Fd[a] += Fu[a] - Fl[a]; }
      const int64_t o = g.at(x, y, k);
      R pc[NP], mc[NM];
#pragma unroll
      for (int a = 0; a < NP; ++a) pc[a] = ph[a][o];
      mc[0] = mu[0][o];
      mc[1] = mu[1][o];
      R A[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) A[a] = R(0.5) * Ss[a] - Fd[a] * (R)P.inv_dx;
      double out[NP];
      phi_cell<R>(P, tab[k], pc, mc, A, out);
#pragma unroll
      for (int a = 0; a < NP; ++a) dst[a * fs + o] = (R)out[a];
    }
  }
}

template <typename R, int D, typename KP, typename CP>
__device__ __forceinline__ void mu_face_at(const KP& P, const CP& C, const PF_GLOBAL R* const* f0,
                                           const PF_GLOBAL R* const* f1,
                                           const PF_GLOBAL R* const* mu, const Geo& g, int xl,
                                           int yl, int zl, R Phi[NM]) {
  if (D == 2 && !g.zface(zl)) {
    Phi[0] = Phi[1] = R(0);
    return;
  }
  R pb[NP], gn[NP], gt1[NP], gt2[NP];
  gather_face<R, D, true>(f0, g, xl, yl, zl, (R)P.inv_dx, (R)P.inv_4dx, pb, gn, gt1, gt2);
  const int xu = D == 0 ? g.xp(xl) : xl;
  const int yu = D == 1 ? g.yp(yl) : yl;
  const int zu = D == 2 ? zl + 1 : zl;
  const int64_t oL = g.at(xl, yl, zl), oU = g.at(xu, yu, zu);
  R dph[3], mL[NM], mU[NM];
#pragma unroll
  for (int a = 0; a < 3; ++a) dph[a] = (f1[a][oL] - f0[a][oL]) + (f1[a][oU] - f0[a][oU]);
#pragma unroll
  for (int q = 0; q < NM; ++q) { mL[q] = mu[q][oL]; mU[q] = mu[q][oU]; }
  mu_face<R, D == 2>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
}

template <typename R>
__global__ __launch_bounds__(kTileThreads) void mu_direct_kernel(DevDomain* const* doms,
                                                                 const int32_t* first, int ndom,
                                                                 int total) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int di = find_domain(first, ndom, item);
    const PF_CONST DevDomain& d = domain_at(doms, di);
    if (!d.active) continue;
    const WorkTile w = decode_item(d, item - first_item(first, di), threadIdx.x);
    if (!w.valid) continue;
    const Geo g = make_geo(d);
    const auto& P = kparams<R>(d);
    const PF_CONST PlaneCoef<R>* tab = to_const(static_cast<const PlaneCoef<R>*>(d.coef));
    const PF_GLOBAL R* src = to_global(static_cast<const R*>(d.copy[d.cur_src]));
    PF_GLOBAL R* dst = to_global(static_cast<R*>(d.copy[d.cur_src ^ 1]));
    const int64_t fs = d.fstride;
    const PF_GLOBAL R* p0[NP] = {src, src + fs, src + 2 * fs, src + 3 * fs};
    const PF_GLOBAL R* mu[NM] = {src + 4 * fs, src + 5 * fs};
    const PF_GLOBAL R* p1[NP] = {dst, dst + fs, dst + 2 * fs, dst + 3 * fs};
    PF_GLOBAL R* mo[NM] = {dst + 4 * fs, dst + 5 * fs};
    const int x = w.x, y = w.y;
    const int xm = g.xm(x), ym = g.ym(y);
    for (int k = w.z0; k < w.z1; ++k) {
      const int64_t o = g.at(x, y, k);
      if (P.mu_frozen) {
        mo[0][o] = mu[0][o];
        mo[1][o] = mu[1][o];
        continue;
      }
      const auto& C = tab[k];
      const auto& Cm = tab[k > 0 ? k - 1 : 0];
      R div[NM] = {R(0), R(0)}, Pu[NM], Pl[NM];
      mu_face_at<R, 0>(P, C, p0, p1, mu, g, x, y, k, Pu);
      mu_face_at<R, 0>(P, C, p0, p1, mu, g, xm, y, k, Pl);
      div[0] += Pu[0] - Pl[0];
      div[1] += Pu[1] - Pl[1];
      mu_face_at<R, 1>(P, C, p0, p1, mu, g, x, y, k, Pu);
      mu_face_at<R, 1>(P, C, p0, p1, mu, g, x, ym, k, Pl);
      div[0] += Pu[0] - Pl[0];
      div[1] += Pu[1] - Pl[1];
      mu_face_at<R, 2>(P, C, p0, p1, mu, g, x, y, k, Pu);
      mu_face_at<R, 2>(P, Cm, p0, p1, mu, g, x, y, k - 1, Pl);
      div[0] = (div[0] + (Pu[0] - Pl[0])) * (R)P.inv_dx;
      div[1] = (div[1] + (Pu[1] - Pl[1])) * (R)P.inv_dx;
      R c0[NP], c1[NP], mc[NM], out[NM];
#pragma unroll
      for (int a = 0; a < NP; ++a) { c0[a] = p0[a][o]; c1[a] = p1[a][o]; }
      mc[0] = mu[0][o];
      mc[1] = mu[1][o];
      mu_cell<R>(P, C, c0, c1, mc, div, out);
      mo[0][o] = out[0];
      mo[1][o] = out[1];
    }
  }
}

// ----------------------------------------------------------------- fill

template <typename R>
__global__ __launch_bounds__(256) void fill_kernel(const DevDomain* dom, const int8_t* phase_map,
                                                   int32_t solid_height, double mu0, double mu1) {
  const DevDomain& d = *dom;
  R* base = static_cast<R*>(d.copy[d.parity]);
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % d.nx);
    const int64_t r = c / d.nx;
    const int y = (int)(r % d.ny);
    const int z = (int)(r / d.ny);
    const int64_t o = (int64_t)z * d.plane + (int64_t)y * d.pitch + x;
    const int ph = z < solid_height ? (int)phase_map[(int64_t)y * d.nx + x] : LQ;
#pragma unroll
    for (int a = 0; a < NP; ++a) base[a * d.fstride + o] = a == ph ? R(1) : R(0);
    base[4 * d.fstride + o] = (R)mu0;
    base[5 * d.fstride + o] = (R)mu1;
  }
}

// Ghost plane nz of both copies for a Dirichlet top: liquid at mu_fill.
template <typename R>
__global__ __launch_bounds__(256) void ghost_kernel(const DevDomain* dom) {
  const DevDomain& d = *dom;
  const int64_t cols = (int64_t)d.nx * d.ny;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cols;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = (int64_t)d.nz * d.plane + (c / d.nx) * d.pitch + c % d.nx;
    for (int cp = 0; cp < 2; ++cp) {
      R* base = static_cast<R*>(d.copy[cp]);
#pragma unroll
      for (int a = 0; a < NP; ++a) base[a * d.fstride + o] = a == LQ ? R(1) : R(0);
      base[4 * d.fstride + o] = (R)d.mu_fill[0];
      base[5 * d.fstride + o] = (R)d.mu_fill[1];
    }
  }
}

// ---------------------------------------------------------- diagnostics

// FP64 partial sums per work group (fixed grid, fixed reduction order, so
// the result is reproducible run to run).  `d` supplies the sizes, the
// element strides of `base` (plane, pitch, fstride), the temperature
// (T0, G, dx, zoff, shifts, v, TE) and the concentration coefficients
// (chi0, chi1, c0, c1): a DevDomain, or a DiagView of fields a caller holds.
template <typename R, typename D>
__device__ __forceinline__ void diag_partial_body(const D& d, const R* base, double t,
                                                  double* partials) {
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  double v[kDiagValues] = {0, 0, 0, 0, 0, 0, 0, __builtin_inf(), -__builtin_inf(), 0};
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % d.nx);
    const int64_t r = c / d.nx;
    const int y = (int)(r % d.ny);
    const int z = (int)(r / d.ny);
    const int64_t o = (int64_t)z * d.plane + (int64_t)y * d.pitch + x;
    double ph[NP], m[NM], S = 0.0, sum = 0.0;
    bool bad = false;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      ph[a] = (double)base[a * d.fstride + o];
      bad |= !__builtin_isfinite(ph[a]);
      S += ph[a] * ph[a];
      sum += ph[a];
      v[2 + a] += ph[a];
      v[7] = fmin(v[7], ph[a]);
      v[8] = fmax(v[8], ph[a]);
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      m[q] = (double)base[(4 + q) * d.fstride + o];
      bad |= !__builtin_isfinite(m[q]);
    }
    v[6] = fmax(v[6], fabs(sum - 1.0));
    v[9] += bad ? 1.0 : 0.0;
    const double T = d.T0 + d.G * ((double)z * d.dx + d.zoff + (double)d.shifts * d.dx - d.v * t);
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      double cq = 0.0;
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        const double chi = d.chi0[a][q] + d.chi1[a][q] * (T - d.TE);
        const double cb = d.c0[a][q] + d.c1[a][q] * (T - d.TE);
        cq += (ph[a] * ph[a] / S) * (chi * m[q] + cb);
      }
      v[q] += cq;
    }
  }
  __shared__ double sh[kDiagValues][256];
#pragma unroll
  for (int i = 0; i < kDiagValues; ++i) sh[i][threadIdx.x] = v[i];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int i = 0; i < kDiagValues; ++i) {
        const double a = sh[i][threadIdx.x], b = sh[i][threadIdx.x + s];
        sh[i][threadIdx.x] = i == 6 || i == 8 ? fmax(a, b) : (i == 7 ? fmin(a, b) : a + b);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < kDiagValues) partials[blockIdx.x * kDiagValues + threadIdx.x] = sh[threadIdx.x][0];
}

template <typename R>
__global__ __launch_bounds__(256) void diag_partial_kernel(const DevDomain* dom, double t,
                                                           double* partials) {
  const DevDomain& d = *dom;
  if (t < 0.0) t = (double)d.step * d.dt;
  diag_partial_body<R>(d, static_cast<const R*>(d.copy[d.parity]), t, partials);
}

// The same sums over fields passed by pointer (the view travels by value).
template <typename R>
__global__ __launch_bounds__(256) void diag_view_kernel(DiagView d, double t, double* partials) {
  diag_partial_body<R>(d, static_cast<const R*>(d.base), t, partials);
}

__global__ __launch_bounds__(64) void diag_final_kernel(const double* partials, int nblocks,
                                                        double* out) {
  const int i = threadIdx.x;
  if (i >= kDiagValues) return;
  double acc = i == 7 ? __builtin_inf() : (i == 8 ? -__builtin_inf() : 0.0);
  for (int b = 0; b < nblocks; ++b) {
    const double x = partials[b * kDiagValues + i];
    acc = i == 6 || i == 8 ? fmax(acc, x) : (i == 7 ? fmin(acc, x) : acc + x);
  }
  out[i] = acc;
}

// --------------------------------------------------------------- launches

hipError_t launch_prologue(const LaunchSet& L, int prec, hipStream_t s) {
  if (prec == 0) {
    prologue_kernel<double><<<L.ndom, 256, 0, s>>>(L.doms, L.ndom);
    coef_kernel<double><<<L.ndom * kCoefBlocks, kCoefThreads, 0, s>>>(L.doms, L.ndom);
  } else {
    prologue_kernel<float><<<L.ndom, 256, 0, s>>>(L.doms, L.ndom);
    coef_kernel<float><<<L.ndom * kCoefBlocks, kCoefThreads, 0, s>>>(L.doms, L.ndom);
  }
  return hipGetLastError();
}

hipError_t launch_window(const LaunchSet& L, int prec, hipStream_t s) {
  // a shift is rare (the front moves a small fraction of a cell per step),
  // so the grid is capped: most launches only read each block's flags
  const int grid = L.total < 1024 ? L.total : 1024;
  if (prec == 0)
    window_kernel<double><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  else
    window_kernel<float><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  return hipGetLastError();
}

hipError_t launch_phi_direct(const LaunchSet& L, int prec, bool aniso, hipStream_t s) {
  const int grid = L.total;
  if (prec == 0) {
    if (aniso)
      phi_direct_kernel<double, true><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
    else
      phi_direct_kernel<double, false><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  } else {
    if (aniso)
      phi_direct_kernel<float, true><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
    else
      phi_direct_kernel<float, false><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  }
  return hipGetLastError();
}

hipError_t launch_mu_direct(const LaunchSet& L, int prec, hipStream_t s) {
  const int grid = L.total;
  if (prec == 0)
    mu_direct_kernel<double><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  else
    mu_direct_kernel<float><<<grid, kTileThreads, 0, s>>>(L.doms, L.first, L.ndom, L.total);
  return hipGetLastError();
}

hipError_t launch_phi(const LaunchSet& L, int prec, bool aniso, int variant, hipStream_t s) {
  if (variant == 1) return launch_phi_tiled(L, prec, aniso, s);
  return launch_phi_direct(L, prec, aniso, s);
}

hipError_t launch_mu(const LaunchSet& L, int prec, int variant, hipStream_t s) {
  if (variant == 1) return launch_mu_tiled(L, prec, s);
  return launch_mu_direct(L, prec, s);
}

hipError_t launch_fill(const DevDomain* dom, int prec, int nx, int ny, int nz,
                       const int8_t* phase_map, int32_t solid_height, double mu0, double mu1,
                       hipStream_t s) {
  const int64_t cells = (int64_t)nx * ny * nz;
  int64_t blocks = (cells + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (prec == 0)
    fill_kernel<double><<<(int)blocks, 256, 0, s>>>(dom, phase_map, solid_height, mu0, mu1);
  else
    fill_kernel<float><<<(int)blocks, 256, 0, s>>>(dom, phase_map, solid_height, mu0, mu1);
  return hipGetLastError();
}

hipError_t launch_ghost(const DevDomain* dom, int prec, int nx, int ny, hipStream_t s) {
  const int64_t cols = (int64_t)nx * ny;
  const int blocks = (int)((cols + 255) / 256 < 1024 ? (cols + 255) / 256 : 1024);
  if (prec == 0)
    ghost_kernel<double><<<blocks, 256, 0, s>>>(dom);
  else
    ghost_kernel<float><<<blocks, 256, 0, s>>>(dom);
  return hipGetLastError();
}

hipError_t launch_diag(const DevDomain* dom, int prec, int nx, int ny, int nz, double t,
                       double* partials, double* out, hipStream_t s) {
  (void)nx;
  (void)ny;
  (void)nz;
  if (prec == 0)
    diag_partial_kernel<double><<<kDiagBlocks, 256, 0, s>>>(dom, t, partials);
  else
    diag_partial_kernel<float><<<kDiagBlocks, 256, 0, s>>>(dom, t, partials);
  diag_final_kernel<<<1, 64, 0, s>>>(partials, kDiagBlocks, out);
  return hipGetLastError();
}

hipError_t launch_diag_view(const DiagView& view, int prec, double t, double* partials,
                            double* out, hipStream_t s) {
  if (prec == 0)
    diag_view_kernel<double><<<kDiagBlocks, 256, 0, s>>>(view, t, partials);
  else
    diag_view_kernel<float><<<kDiagBlocks, 256, 0, s>>>(view, t, partials);
  diag_final_kernel<<<1, 64, 0, s>>>(partials, kDiagBlocks, out);
  return hipGetLastError();
}

}  // namespace pfk
