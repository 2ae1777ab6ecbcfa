// pf_device.h -- device-side data structures and model arithmetic of the
// phase-field stepper (Bauer et al., SC'15, arXiv:1506.01684).
//
// Model (Sec. 2): four order parameters phi_a on the Gibbs simplex (phases
// 0..2 solid, 3 liquid), two chemical potentials mu_i, frozen temperature
// T(z,t) = T0 + G (z + zoff - v t).  The phi equation (Eqs. (1)-(2)) is
// discretised on cell faces: every face carries the normal component F_a of
// da/d(grad phi_a) and its share S_a of da/dphi_a; the cell combines its six
// faces.  The mu equation (Eq. (3)) is written in flux form: every face
// carries Phi_i = M_i d mu_i - J_i with the anti-trapping current of Eq. (4);
// the cell combines the divergence with exact-difference source terms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Address spaces of gfx9: 1 = global (vector memory), 4 = constant (read
// only for the duration of a kernel; loads with a uniform address become
// scalar loads).  Field pointers are cast to global so loads are not flat
// loads; descriptors and per-plane coefficient tables, written only by other
// kernels, are read through the constant space.
#define PF_GLOBAL __attribute__((address_space(1)))
#define PF_CONST __attribute__((address_space(4)))

namespace pfk {

template <typename T>
__device__ __forceinline__ const PF_CONST T* to_const(const T* p) {
  return (const PF_CONST T*)(p);
}
template <typename T>
__device__ __forceinline__ PF_GLOBAL T* to_global(T* p) {
  return (PF_GLOBAL T*)(p);
}

constexpr int NP = 4;   // phases
constexpr int NM = 2;   // chemical potentials
constexpr int LQ = 3;   // liquid index
constexpr int NPAIR = 6;
constexpr int NFIELD = 6;  // phi_0..phi_3, mu_0, mu_1 in one copy

// Per-step counts of the tiled sweeps, after the item words of jfree: the
// light items (no anti-trapping face), the items the phi bulk shortcut
// keeps, the items whose mu-sweep reads mu alone, and the kept items whose
// phi the bulk shortcut had to copy (not already in both copies).
// Increments of one address are serialised, so each count is spread over
// kCountSlots words on 128-byte lines of their own (the work item's number
// picks the slot).
constexpr int kCountKinds = 4, kCountSlots = 8, kCountStride = 32;  // stride in words
constexpr int kCountLight = 0, kCountFixed = 1, kCountPure = 2, kCountCopied = 3;
constexpr int kCountWords = kCountKinds * kCountSlots * kCountStride;
__host__ __device__ inline int64_t count_base(int64_t nitems) {  // word offset in jfree
  return (nitems + kCountStride - 1) / kCountStride * kCountStride;
}
__host__ __device__ inline int64_t count_word(int kind, int slot) {
  return (int64_t)(kind * kCountSlots + slot) * kCountStride;
}

// pair index of (a,b), a < b: (0,1)=0 (0,2)=1 (0,3)=2 (1,2)=3 (1,3)=4 (2,3)=5
__host__ __device__ constexpr int pair_index(int a, int b) {
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

// Kernel-side parameters in the arithmetic type R.
template <typename R>
struct KParams {
  R g1[NPAIR];     // gamma_ab
  R g2[NPAIR];     // 2 gamma_ab
  R g16[NPAIR];    // 16/pi^2 gamma_ab (pair part of d omega / d phi)
  R delta[NPAIR];  // cubic anisotropy strength
  R ac0[NPAIR];    // 1 - 3 delta
  R d4[NPAIR];     // 4 delta
  R d16[NPAIR];    // 16 delta
  R gamma3;        // triple coefficient
  R rate[NP];      // dt / (tau_a eps)
  R inv_dx, inv_4dx;
  R dt, half_inv_dt;  // dt, 1/(2 dt)
  R pieps4;           // pi eps / 4
  int32_t aniso, antitrap, mu_frozen, shortcuts;
  int32_t aniso_mask;  // bit i set: pair i has delta > 0
  int32_t pad[3];
};

// Per z-plane coefficients of one step, all evaluated in FP64 and then
// rounded to R (Sec. 3.3: everything that depends only on the analytic
// temperature is computed once per z slice).
template <typename R>
struct PlaneCoef {
  R epsT, Toe;          // eps T, T/eps at T^n_k
  R chi[NP][NM];        // chi_ai(T^n_k)
  R cbar[NP][NM];       // cbar_ai(T^n_k)
  R wbar[NP];           // omega_bar_a(T^n_k)
  R Dchi[NP][NM];       // D_a chi_ai(T^n_k)          (x/y faces)
  R dchiL[3][NM];       // chi_li - chi_ai at T^n_k    (x/y faces, a < 3)
  R dcbL[3][NM];        // cbar_li - cbar_ai at T^n_k
  R DchiZ[NP][NM];      // the same three at T^n_{k+1/2} (z face)
  R dchiLZ[3][NM];
  R dcbLZ[3][NM];
  R chi1[NP][NM];       // chi_ai(T^{n+1}_k)
  R dchi[NP][NM];       // chi(T^{n+1}_k) - chi(T^n_k)  (difference in FP64)
  R dcbar[NP][NM];      // cbar(T^{n+1}_k) - cbar(T^n_k)
  // for the mu-sweep of cells whose phi^n, phi^{n+1} and neighbours are all
  // e_a, computed by the same functions as in the general face and cell
  // stages (mu_face_m, mu_cell_h, mu_cell_chi), so bitwise the same values:
  R Mp[NP][NM];         // mu_face_m at pb = e_a, x/y faces
  R MpZ[NP][NM];        // mu_face_m at pb = e_a, z face
  R rchip[NP][NM];      // rcp_ of mu_cell's chi sum at phi^{n+1} = e_a
  int32_t pure_fixed;   // bit a: a pure-a cell with zero face terms maps to itself
  int32_t chunk_fixed;  // first plane of a z chunk: pure_fixed of all its planes
};

// Device-resident descriptor of one domain.
struct DevDomain {
  int32_t nx, ny, nz, pitch;  // cells; row stride in elements
  int64_t plane, fstride;     // plane stride; field stride (elements)
  int32_t tx, ty, zc;         // tile: tx * ty threads, zc planes per item
  int32_t ntx, nty, nzc;      // tiles per axis
  int32_t xmode, rs;          // XCD y-slab order (1) with rs tile rows per XCD, or plain (0)
  int32_t prec;               // 0 = FP64, 1 = FP32
  int32_t active;             // set by the prologue for the current step
  int64_t step;               // index n of the next step (state time n dt)
  int32_t parity;             // copy that holds the current state
  int32_t cur_src;            // prologue: source copy of the running step
  int64_t cur_step;           // prologue: index of the running step
  int64_t steps_left;         // < 0: unlimited
  int32_t window_z;           // moving-window plane (0 = off)
  int32_t shift_now;          // prologue: this step starts with a window shift
  int64_t shifts;             // window shifts so far (z origin = zoff + shifts dx)
  int32_t shift_src;          // prologue: copy the shift reads (it writes cur_src)
  int32_t top_bc;             // 1: Dirichlet top (ghost plane nz held at liquid, mu_fill)
  double mu_fill[NM];         // mu of the liquid plane a shift adds / of the ghost plane
  void* copy[2];              // base of each 6-field copy
  void* coef;                 // PlaneCoef<R>[nz] of the running step
  void* jfree;                // uint32 per work item of the tiled sweeps, then the counts
  int32_t nitems;             // work items of the tiled sweeps (index of those counts)
  int32_t pflag_ok[2];        // pflag[c] describes the state held in copy c
  void* pflag[2];             // uint8 per tile and z chunk [iz][iy][ix]: the phase all
                              // cells of the chunk hold purely in copy c, 0xFF if none
  void* pends[2];             // uint8 per chunk, same order: the pure phase of its
                              // bottom plane (low nibble) and top plane (high), 0xF if none
  double dt, dx;
  double eps, TE, T0, G, v, zoff;
  double chi0[NP][NM], chi1[NP][NM], c0[NP][NM], c1[NP][NM];
  double w0[NP], w1[NP], D[NP];
  KParams<double> kp64;
  KParams<float> kp32;
};

template <typename R, typename DD>
__device__ __forceinline__ const auto& kparams(const DD& d) {
  if constexpr (sizeof(R) == 8) return d.kp64;
  else return d.kp32;
}

// ------------------------------------------------------------ math helpers
//
// fma_: a*b+c with one rounding.
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
//
// FP64: hardware reciprocal / reciprocal square root refined by two Newton
// steps (relative error about one ulp); FP32: the hardware instructions
// (about one ulp).  Arguments are positive and normal wherever they are used.

__device__ __forceinline__ double rcp_(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsq_(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double e = __builtin_fma(-x * r, r, 1.0);
  r = __builtin_fma(0.5 * r, e, r);
  e = __builtin_fma(-x * r, r, 1.0);
  return __builtin_fma(0.5 * r, e, r);
}
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }

// --------------------------------------------------------- phi face stage

// Cubic-anisotropic pair term: X = d(ac(q)^2 |q|^2)/dq
//   = 2 ac [ ac q + 16 delta |q| (qhat^3 - P qhat) ],  P = sum qhat_i^4,
// with X = 2 q when |q|^2 <= 1e-30.  Only the component along the face
// normal D is needed; with u_i = q_i^2 / |q|^2 (so P = sum u_i^2) it is
//   X.e_D = 2 ac q_D [ ac + 16 delta (u_D - P) ],  ac = (1 - 3 delta) + 4 delta P,
// which needs one reciprocal and no square root, and every u_i <= 1 keeps
// the FP32 evaluation in range.  ac0 = 1 - 3 delta, d4 = 4 delta,
// d16 = 16 delta.
template <typename R, int D>
__device__ __forceinline__ R aniso_Xd(R qx, R qy, R qz, R ac0, R d4, R d16) {
  const R x2 = qx * qx, y2 = qy * qy, z2 = qz * qz;
  const R qq = x2 + y2 + z2;
  const R r = rcp_(qq > R(1e-30) ? qq : R(1));
  const R ux = x2 * r, uy = y2 * r, uz = z2 * r;
  const R P = ux * ux + uy * uy + uz * uz;
  const R ac = ac0 + d4 * P;
  const R qd = D == 0 ? qx : (D == 1 ? qy : qz);
  const R ud = D == 0 ? ux : (D == 1 ? uy : uz);
  const R X = R(2) * ac * qd * (ac + d16 * (ud - P));
  // branch-free guard: with the exact shortcuts most faces reaching here
  // are interface faces, where a branch would only add mask handling
  return qq > R(1e-30) ? X : R(2) * qd;
}

// Face stage of the phi-sweep on a face with normal D.
//  pb[a]  face average of phi_a
//  gn[a]  normal difference (phi_a,U - phi_a,L)/dx
//  gt1/gt2 tangential components (only read when ANISO)
// Outputs F_a = sum_{b!=a} gamma_ab (-pb_b) X_ab.e_D  and
//         S_a = sum_{b!=a} gamma_ab  X_ab.e_D (gn_b),  X_ba = -X_ab.
template <typename R, bool ANISO, int D, typename KP>
__device__ __forceinline__ void phi_face(const KP& P, const R pb[NP], const R gn[NP],
                                         const R gt1[NP], const R gt2[NP], R F[NP], R S[NP]) {
#pragma unroll
  for (int a = 0; a < NP; ++a) F[a] = S[a] = R(0);
#pragma unroll
  for (int a = 0; a < NP; ++a) {
#pragma unroll
    for (int b = a + 1; b < NP; ++b) {
      const int pi = pair_index(a, b);
      R Y;  // gamma_ab X_ab.e_D
      // pairs without anisotropy take X.e_D = 2 q.e_D (a uniform branch)
      if (ANISO && ((P.aniso_mask >> pi) & 1)) {
        // full generalised gradient q = pb_a grad phi_b - pb_b grad phi_a
        R qn = pb[a] * gn[b] - pb[b] * gn[a];
        R q1 = pb[a] * gt1[b] - pb[b] * gt1[a];
        R q2 = pb[a] * gt2[b] - pb[b] * gt2[a];
        R qx, qy, qz;
        if constexpr (D == 0) { qx = qn; qy = q1; qz = q2; }
        else if constexpr (D == 1) { qx = q1; qy = qn; qz = q2; }
        else { qx = q1; qy = q2; qz = qn; }
        Y = (R)P.g1[pi] * aniso_Xd<R, D>(qx, qy, qz, (R)P.ac0[pi], (R)P.d4[pi], (R)P.d16[pi]);
      } else {
        Y = (R)P.g2[pi] * (pb[a] * gn[b] - pb[b] * gn[a]);
      }
      F[a] -= pb[b] * Y;
      F[b] += pb[a] * Y;
      S[a] += Y * gn[b];
      S[b] -= Y * gn[a];
    }
  }
}

// Contributions of one phi face to the A_a of its two cells (A_a = half the
// sum of the six face shares minus the flux differences over dx): to the
// cell below the face, whose upper face it is, P_a = S_a/2 - F_a/dx; to the
// cell above, Q_a = S_a/2 + F_a/dx.  Each rounding is spelled out.
template <typename R>
__device__ __forceinline__ void face_pq(const R F[NP], const R S[NP], R inv_dx, R Pv[NP], R Qv[NP]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    const R h = R(0.5) * S[a];
    Pv[a] = fma_(-F[a], inv_dx, h);
    Qv[a] = fma_(F[a], inv_dx, h);
  }
}

// Exact shortcut tests (the paper's shortcuts, Sec. 3.3, restricted to work
// whose result is known exactly).
//
// A phi face whose normal differences all vanish carries F = S = 0 exactly:
// then q_ab.e_D = 0 for every pair, so X_ab.e_D = 0 also on anisotropic
// pairs (q_hat.e_D = 0), and S_a sums Y gn_b = 0.
template <typename R>
__device__ __forceinline__ bool zero_normal(const R gn[NP]) {
  return gn[0] == R(0) && gn[1] == R(0) && gn[2] == R(0) && gn[3] == R(0);
}

// A pure cell (phi = e_a exactly) with A = 0 (as when its faces vanish) has a zero
// driving force and obstacle derivative 16/pi^2 gamma_ab for the absent
// phases; when its plane marks e_a as a fixed point of the Euler step and
// the projection (fixed_mask bit a), its new value is e_a again.
template <typename R>
__device__ __forceinline__ bool pure_cell_fixed(const R ph[NP], const R A[NP], int fixed_mask) {
#pragma unroll
  for (int a = 0; a < NP; ++a)
    if (A[a] != R(0)) return false;
  const int a1 = ph[0] == R(1) ? 0 : (ph[1] == R(1) ? 1 : (ph[2] == R(1) ? 2 : (ph[3] == R(1) ? 3 : -1)));
  if (a1 < 0) return false;
  int nonzero = 0;
#pragma unroll
  for (int b = 0; b < NP; ++b) nonzero += ph[b] != R(0);
  return nonzero == 1 && ((fixed_mask >> a1) & 1);
}

// ------------------------------------------------------------ projection

// Euclidean projection of y onto {x >= 0, sum x = 1} followed by
// renormalisation, in FP64: sort descending, rho = largest j with
// j u_j > s_j - 1 (u_j - (s_j - 1)/j > 0 multiplied by j > 0), threshold
// theta = (s_rho - 1)/rho, clip, divide by the sum.
__device__ __forceinline__ void project_simplex(const double y[NP], double x[NP]) {
  double u0 = y[0], u1 = y[1], u2 = y[2], u3 = y[3];
#define PF_CSWAP(a, b)      \
  {                         \
    double hi = fmax(a, b); \
    double lo = fmin(a, b); \
    a = hi;                 \
    b = lo;                 \
  }
  PF_CSWAP(u0, u1);
  PF_CSWAP(u2, u3);
  PF_CSWAP(u0, u2);
  PF_CSWAP(u1, u3);
  PF_CSWAP(u1, u2);
#undef PF_CSWAP
  const double s1 = u0, s2 = s1 + u1, s3 = s2 + u2, s4 = s3 + u3;
  double theta = s1 - 1.0;
  if (2.0 * u1 > s2 - 1.0) theta = (s2 - 1.0) * 0.5;
  if (3.0 * u2 > s3 - 1.0) theta = (s3 - 1.0) * (1.0 / 3.0);
  if (4.0 * u3 > s4 - 1.0) theta = (s4 - 1.0) * 0.25;
  double xs[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) xs[a] = fmax(y[a] - theta, 0.0);
  const double inv = rcp_(((xs[0] + xs[1]) + xs[2]) + xs[3]);
#pragma unroll
  for (int a = 0; a < NP; ++a) x[a] = xs[a] * inv;
}

// -------------------------------------------------------- phi cell stage

// Cell stage of the phi-sweep (Eqs. (1)-(2)): A_a from the faces, the
// obstacle derivative, the driving force (2 phi_a/S)(psi_a - sum h_b psi_b),
// rhs_a = eps T A_a + (T/eps) omega'_a + psi'_a, Lagrange mean over the four
// phases, explicit Euler, projection.
//   A[a] = 1/2 sum over the six faces of S - sum over directions of
//          (F_up - F_low) / dx
template <typename R, typename KP, typename CP>
__device__ __forceinline__ void phi_cell(const KP& P, const CP& C, const R ph[NP], const R mu[NM],
                                         const R A[NP], double out[NP]) {
  R S = ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2] + ph[3] * ph[3];
  R invS = rcp_(S);
  R psi[NP], psibar = R(0);
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    R quad = (R)C.chi[a][0] * mu[0] * mu[0] + (R)C.chi[a][1] * mu[1] * mu[1];
    R lin = (R)C.cbar[a][0] * mu[0] + (R)C.cbar[a][1] * mu[1];
    psi[a] = R(-0.5) * quad - lin + (R)C.wbar[a];
    psibar += (ph[a] * ph[a]) * psi[a];
  }
  psibar *= invS;
  R rhs[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    R dpsi = (R(2) * ph[a] * invS) * (psi[a] - psibar);
    R pair = R(0), triple = R(0);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      if (b == a) continue;
      pair += (R)P.g16[a < b ? pair_index(a, b) : pair_index(b, a)] * ph[b];
#pragma unroll
      for (int e = b + 1; e < NP; ++e)
        if (e != a) triple += ph[b] * ph[e];
    }
    R domega = pair + (R)P.gamma3 * triple;
    rhs[a] = (R)C.epsT * A[a] + (R)C.Toe * domega + dpsi;
  }
  R mean = R(0.25) * (((rhs[0] + rhs[1]) + rhs[2]) + rhs[3]);
  double y[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) y[a] = (double)(ph[a] - (R)P.rate[a] * (rhs[a] - mean));
  project_simplex(y, out);
}

// --------------------------------------------------------- mu face stage

// Face stage of the mu-sweep on a face with normal D (Eq. (3) flux and the
// normal component of Eq. (4)); ZF selects the coefficients at T(k+1/2):
//   M_i = sum_a D_a pb_a chi_ai(T_f),  diff_i = M_i (mu_i,U - mu_i,L)/dx
//   J_i = (pi eps/4) sum_{a<3} w_a rate_a (n_a.n_l)(n_a.e_D) dc_ai
//   w_a = sqrt(pb_a pb_l) pb_l / sum pb^2  (= g_a h_l / sqrt(phi_a phi_l))
//   (n_a.n_l)(n_a.e_D) = (g_a.g_l) g_a,D / (|g_a|^2 |g_l|), 0 if a gradient is 0
//   dc_ai = (chi_li - chi_ai) mubar_i + (cbar_li - cbar_ai)
// pb: face average of phi^n; gn/gt1/gt2: normal and tangential face
// gradient of phi^n; dph: (phi^{n+1}-phi^n)_L + (...)_U per solid phase;
// mL/mU: mu^n at the face cells.
// Diffusive part M_i (mu_i,U - mu_i,L)/dx of the face flux.  Here and in
// mu_cell every rounding step is written out (fused where fma_ says so) and
// contraction is off, so that each kernel evaluating these formulas rounds
// them identically wherever they are inlined.
template <typename R, bool ZF, typename CP>
__device__ __forceinline__ void mu_face_m(const CP& C, const R pb[NP], R M[NM]) {
#pragma clang fp contract(off)
  M[0] = (R)(ZF ? C.DchiZ[0][0] : C.Dchi[0][0]) * pb[0];
  M[1] = (R)(ZF ? C.DchiZ[0][1] : C.Dchi[0][1]) * pb[0];
#pragma unroll
  for (int a = 1; a < NP; ++a) {
    M[0] = fma_(ZF ? C.DchiZ[a][0] : C.Dchi[a][0], pb[a], M[0]);
    M[1] = fma_(ZF ? C.DchiZ[a][1] : C.Dchi[a][1], pb[a], M[1]);
  }
}
template <typename R>
__device__ __forceinline__ R mu_face_flux(R M, R mL, R mU, R inv_dx) {
#pragma clang fp contract(off)
  return M * (mU - mL) * inv_dx;
}
template <typename R, bool ZF, typename KP, typename CP>
__device__ __forceinline__ void mu_face_diff(const KP& P, const CP& C, const R pb[NP],
                                             const R mL[NM], const R mU[NM], R Phi[NM]) {
  R M[NM];
  mu_face_m<R, ZF>(C, pb, M);
  Phi[0] = mu_face_flux<R>(M[0], mL[0], mU[0], (R)P.inv_dx);
  Phi[1] = mu_face_flux<R>(M[1], mL[1], mU[1], (R)P.inv_dx);
}

// The anti-trapping current vanishes exactly unless some solid phase and the
// liquid are both present on the face (w_a = 0 when pb_a pb_l <= 0).
template <typename R>
__device__ __forceinline__ bool mu_face_needs_j(const R pb[NP]) {
  return pb[0] * pb[LQ] > R(0) || pb[1] * pb[LQ] > R(0) || pb[2] * pb[LQ] > R(0);
}

// Anti-trapping part: subtracts (pi eps/4) J_i from Phi_i.
template <typename R, bool ZF, typename KP, typename CP>
__device__ __forceinline__ void mu_face_j(const KP& P, const CP& C, const R pb[NP], const R gn[NP],
                                          const R gt1[NP], const R gt2[NP], const R dph[3],
                                          const R mL[NM], const R mU[NM], R Phi[NM]) {
  const R mb0 = R(0.5) * (mL[0] + mU[0]), mb1 = R(0.5) * (mL[1] + mU[1]);
  const R gl2 = gn[LQ] * gn[LQ] + gt1[LQ] * gt1[LQ] + gt2[LQ] * gt2[LQ];
  if (!(gl2 > R(0))) return;
  const R pl = pb[LQ];
  const R Sb = pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2] + pl * pl;
  const R base = pl * rcp_(Sb) * rsq_(gl2) * (R)P.half_inv_dt;
  R J0 = R(0), J1 = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R prod = pb[a] * pl;
    R ga2 = gn[a] * gn[a] + gt1[a] * gt1[a] + gt2[a] * gt2[a];
    if (prod > R(0) && ga2 > R(0)) {
      R dot = gn[a] * gn[LQ] + gt1[a] * gt1[LQ] + gt2[a] * gt2[LQ];
      R coef = (prod * rsq_(prod)) * base * dph[a] * (dot * gn[a]) * rcp_(ga2);
      const R dc0 = (R)(ZF ? C.dchiLZ[a][0] : C.dchiL[a][0]) * mb0 +
                    (R)(ZF ? C.dcbLZ[a][0] : C.dcbL[a][0]);
      const R dc1 = (R)(ZF ? C.dchiLZ[a][1] : C.dchiL[a][1]) * mb1 +
                    (R)(ZF ? C.dcbLZ[a][1] : C.dcbL[a][1]);
      J0 += coef * dc0;
      J1 += coef * dc1;
    }
  }
  Phi[0] -= (R)P.pieps4 * J0;
  Phi[1] -= (R)P.pieps4 * J1;
}

// Whole face flux Phi_i = M_i d mu_i - (pi eps/4) J_i.
template <typename R, bool ZF, typename KP, typename CP>
__device__ __forceinline__ void mu_face(const KP& P, const CP& C, const R pb[NP], const R gn[NP],
                                        const R gt1[NP], const R gt2[NP], const R dph[3],
                                        const R mL[NM], const R mU[NM], R Phi[NM]) {
  mu_face_diff<R, ZF>(P, C, pb, mL, mU, Phi);
  if (P.antitrap && mu_face_needs_j(pb)) mu_face_j<R, ZF>(P, C, pb, gn, gt1, gt2, dph, mL, mU, Phi);
}

// ---------------------------------------------------------- mu cell stage

// Cell stage of the mu-sweep: c^{n+1} - c^n = dt div(Phi) is solved for
// mu^{n+1} with c = sum_a h_a (chi_a mu + cbar_a):
//   src_i = sum_a (h1_a - h0_a)(chi_ai mu_i + cbar_ai - cbar_li)
//         + sum_a h1_a (dchi_ai mu_i + dcbar_ai)
//   mu_i^{n+1} = mu_i + (dt div_i - src_i) / sum_a h1_a chi_ai(T^{n+1})
// h_a = phi_a^2 / sum_b phi_b^2 of one cell.
template <typename R>
__device__ __forceinline__ void mu_cell_h(const R p[NP], R h[NP]) {
#pragma clang fp contract(off)
  R S = p[0] * p[0];
#pragma unroll
  for (int a = 1; a < NP; ++a) S = fma_(p[a], p[a], S);
  const R i = rcp_(S);
#pragma unroll
  for (int a = 0; a < NP; ++a) h[a] = p[a] * p[a] * i;
}
// src_i for component q; dh = h1 - h0, cd_a = cbar_ai - cbar_li.
template <typename R, typename CP>
__device__ __forceinline__ R mu_cell_src(const CP& C, int q, const R dh[NP], const R h1[NP], R mu,
                                         const R cd[NP]) {
#pragma clang fp contract(off)
  R src = R(0);
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    const R ca = fma_(C.chi[a][q], mu, cd[a]);
    const R ta = fma_(C.dchi[a][q], mu, C.dcbar[a][q]);
    src = fma_(dh[a], ca, src);
    src = fma_(h1[a], ta, src);
  }
  return src;
}
// src of a cell with phi^n = phi^{n+1} = e_a (h_a = ha = 1, h1 - h0 = +0):
// the one term of the sum above that is not a finite value times +0.
template <typename R>
__device__ __forceinline__ R mu_pure_src(R ha, R dchi_a, R dcbar_a, R mu) {
#pragma clang fp contract(off)
  return fma_(ha, fma_(dchi_a, mu, dcbar_a), R(0));
}
// sum_a h1_a chi_ai(T^{n+1}) for component q.
template <typename R, typename CP>
__device__ __forceinline__ R mu_cell_chi(const CP& C, int q, const R h1[NP]) {
#pragma clang fp contract(off)
  R chi = R(0);
#pragma unroll
  for (int a = 0; a < NP; ++a) chi = fma_(h1[a], C.chi1[a][q], chi);
  return chi;
}
template <typename R, typename KP>
__device__ __forceinline__ R mu_cell_out(const KP& P, R div, R src, R rchi, R mu) {
#pragma clang fp contract(off)
  return fma_(fma_(P.dt, div, -src), rchi, mu);
}
template <typename R, typename KP, typename CP>
__device__ __forceinline__ void mu_cell(const KP& P, const CP& C, const R p0[NP], const R p1[NP],
                                        const R mu[NM], const R div[NM], R out[NM]) {
#pragma clang fp contract(off)
  R h0[NP], h1[NP], dh[NP];
  mu_cell_h<R>(p0, h0);
  mu_cell_h<R>(p1, h1);
#pragma unroll
  for (int a = 0; a < NP; ++a) dh[a] = h1[a] - h0[a];
#pragma unroll
  for (int q = 0; q < NM; ++q) {
    const R cref = (R)C.cbar[LQ][q];
    R cd[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) cd[a] = (R)C.cbar[a][q] - cref;
    const R src = mu_cell_src<R>(C, q, dh, h1, mu[q], cd);
    out[q] = mu_cell_out<R>(P, div[q], src, rcp_(mu_cell_chi<R>(C, q, h1)), mu[q]);
  }
}

}  // namespace pfk
