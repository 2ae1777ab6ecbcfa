/*
 * pf_oracle.c -- plain FP64 CPU oracle of the grand-potential multi-phase-field
 * time step of Bauer et al. (SC'15, arXiv:1506.01684).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * What it computes, in the paper's notation (Sec. 2 "Model", Sec. 2.1,
 * Algorithm 1):
 *   phi-kernel  Eq. (1)+(2): d phi_a/dt = -(1/(tau_a eps)) (rhs_a - mean_b rhs_b),
 *               rhs_a = eps T (da/dphi_a - div da/dgrad phi_a)
 *                     + (T/eps) domega/dphi_a + dpsi/dphi_a,
 *               explicit Euler, then projection back onto the Gibbs simplex
 *               (the simplex constraint of Sec. 2; the projection of Sec. 5.1.1).
 *   mu-kernel   Eq. (3): dmu/dt = (dc/dmu)^-1 ( -dc/dphi dphi/dt - dc/dT dT/dt
 *               + div(M grad mu) - div J_at ), J_at from Eq. (4), reading
 *               mu_src, phi_src and phi_dst exactly as Algorithm 1 does.
 *   frozen temperature T(z,t) = T0 + G (z - v t) (Sec. 2 and Sec. 3.3).
 *
 * The paper fixes the PDEs but not the free-energy forms or the finite-
 * difference stencils.  The readings taken here are:
 *   - sign of Eq. (1): minus (energy descent);
 *   - a = sum_{a<b} gamma_ab ac(q_ab)^2 |q_ab|^2, q_ab = phi_a grad phi_b -
 *     phi_b grad phi_a, cubic ac(q) = 1 - delta (3 - 4 sum_i (q_i/|q|)^4);
 *   - multi-obstacle omega = 16/pi^2 sum gamma_ab phi_a phi_b
 *     + gamma3 sum phi_a phi_b phi_c;
 *   - quadratic grand potentials psi_a = -1/2 sum_i chi_ai mu_i^2
 *     - sum_i cbar_ai mu_i + omega_bar_a, all coefficients linear in T;
 *   - h_a = phi_a^2 / sum_b phi_b^2 everywhere, g_a = phi_a;
 *   - mobility M_i = sum_a D_a phi_a chi_ai(T);
 *   - staggered (face-centred) differences: each face flux uses the face
 *     average, the normal difference and 4-point tangential averages;
 *   - mu-sweep geometry from phi^n, dphi/dt from phi^{n+1}-phi^n, h and chi
 *     from phi^{n+1}, source terms written as exact differences so that the
 *     total concentration changes only by the flux divergence;
 *   - projection: Euclidean projection onto the simplex, then
 *     renormalisation;
 *   - boundaries: periodic in x and y, zero-flux mirror in z.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NP ORC_NPHASE
#define NM ORC_NMU
#define LQ ORC_LIQ

static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ grid */

static int wrap_index(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

/* Zero-gradient mirror for one ghost layer: -1 -> 0, nz -> nz-1. */
static int mirror_index(int k, int nz) {
  if (k < 0) return 0;
  if (k >= nz) return nz - 1;
  return k;
}

static size_t ncells(const orc_grid* g) {
  return (size_t)g->nx * (size_t)g->ny * (size_t)g->nz;
}

static size_t cell(const orc_grid* g, int i, int j, int k) {
  i = wrap_index(i, g->nx);
  j = wrap_index(j, g->ny);
  k = mirror_index(k, g->nz);
  return ((size_t)k * (size_t)g->ny + (size_t)j) * (size_t)g->nx + (size_t)i;
}

static const int UNIT[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* Value of field f (a pointer to one scalar field) at (i,j,k)+s*e_d. */
static double at(const orc_grid* g, const double* f, int i, int j, int k,
                 int d, int s) {
  return f[cell(g, i + s * UNIT[d][0], j + s * UNIT[d][1], k + s * UNIT[d][2])];
}

/* ------------------------------------------------------- model functions */

uint64_t orc_splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double orc_temperature(const orc_params* p, const orc_grid* g, double zc,
                       double t) {
  return p->T0 + p->G * (zc * g->dx + p->zoff - p->v * t);
}

static double chi_of(const orc_params* p, int a, int i, double T) {
  return p->chi0[a][i] + p->chi1[a][i] * (T - p->TE);
}

static double cbar_of(const orc_params* p, int a, int i, double T) {
  return p->c0[a][i] + p->c1[a][i] * (T - p->TE);
}

static double wbar_of(const orc_params* p, int a, double T) {
  return p->w0[a] + p->w1[a] * (T - p->TE);
}

/* Grand potential of phase a (quadratic in mu). */
static double psi_of(const orc_params* p, int a, const double mu[2], double T) {
  double quad = chi_of(p, a, 0, T) * mu[0] * mu[0] +
                chi_of(p, a, 1, T) * mu[1] * mu[1];
  double lin = cbar_of(p, a, 0, T) * mu[0] + cbar_of(p, a, 1, T) * mu[1];
  return -0.5 * quad - lin + wbar_of(p, a, T);
}

/* Concentration of component i in phase a: c = -dpsi/dmu_i. */
static double conc_of(const orc_params* p, int a, int i, const double mu[2],
                      double T) {
  return chi_of(p, a, i, T) * mu[i] + cbar_of(p, a, i, T);
}

/* Interpolation h_a = phi_a^2 / sum_b phi_b^2 for all four phases. */
static void interp_h(const double ph[4], double h[4]) {
  double s = ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2] + ph[3] * ph[3];
  for (int a = 0; a < NP; ++a) h[a] = ph[a] * ph[a] / s;
}

static int anisotropy_active(const orc_params* p) {
  for (int a = 0; a < NP; ++a)
    for (int b = a + 1; b < NP; ++b)
      if (p->delta[a][b] != 0.0) return 1;
  return 0;
}

double orc_stability_bound(const orc_params* p, const orc_grid* g) {
  double tau_min = p->tau[0], gmax = 0.0, dmax = 0.0;
  for (int a = 0; a < NP; ++a) {
    if (p->tau[a] < tau_min) tau_min = p->tau[a];
    for (int b = a + 1; b < NP; ++b) {
      if (p->gamma[a][b] > gmax) gmax = p->gamma[a][b];
      if (p->delta[a][b] > dmax) dmax = p->delta[a][b];
    }
  }
  double Tb = orc_temperature(p, g, 0.0, 0.0);
  double Tt = orc_temperature(p, g, (double)(g->nz - 1), 0.0);
  double Tmax = Tb > Tt ? Tb : Tt;
  double Tmin = Tb > Tt ? Tt : Tb;
  /* Phase-field part: two-phase linearisation has diffusivity 2 gamma T/tau;
   * the 7-point explicit limit is dx^2/(6 D); cubic anisotropy stiffens it by
   * (1+delta)(1+15 delta). */
  double kappa = (1.0 + dmax) * (1.0 + 15.0 * dmax);
  double dt_phi = g->dx * g->dx * tau_min / (12.0 * gmax * Tmax * kappa);
  /* Chemical part: effective diffusivity at most max(D chi)/min(chi). */
  double chi_min = INFINITY, dchi_max = 0.0;
  for (int a = 0; a < NP; ++a)
    for (int i = 0; i < NM; ++i) {
      double Ts[2] = {Tmin, Tmax};
      for (int s = 0; s < 2; ++s) {
        double c = chi_of(p, a, i, Ts[s]);
        if (c < chi_min) chi_min = c;
        if (p->D[a] * c > dchi_max) dchi_max = p->D[a] * c;
      }
    }
  double dt_mu = g->dx * g->dx * chi_min / (6.0 * dchi_max);
  return dt_phi < dt_mu ? dt_phi : dt_mu;
}

/* ------------------------------------------------------------ projection */

void orc_project(const double y[4], double x[4]) {
  double u[4] = {y[0], y[1], y[2], y[3]};
  /* sort descending (insertion sort) */
  for (int a = 1; a < 4; ++a) {
    double val = u[a];
    int b = a - 1;
    while (b >= 0 && u[b] < val) {
      u[b + 1] = u[b];
      --b;
    }
    u[b + 1] = val;
  }
  /* rho = largest j with u_j - (s_j - 1)/j > 0; theta = (s_rho - 1)/rho */
  double s = 0.0, s_rho = u[0];
  int rho = 1;
  for (int j = 0; j < 4; ++j) {
    s = s + u[j];
    if (u[j] - (s - 1.0) / (double)(j + 1) > 0.0) {
      rho = j + 1;
      s_rho = s;
    }
  }
  double theta = (s_rho - 1.0) / (double)rho;
  double xs[4];
  for (int a = 0; a < 4; ++a) {
    double v = y[a] - theta;
    xs[a] = v > 0.0 ? v : 0.0;
  }
  double sum = ((xs[0] + xs[1]) + xs[2]) + xs[3];
  for (int a = 0; a < 4; ++a) x[a] = xs[a] / sum;
}

/* --------------------------------------------------- gradient energy (a) */

void orc_aniso_X(const double q[3], double delta, double X[3]) {
  if (delta == 0.0) {
    for (int c = 0; c < 3; ++c) X[c] = 2.0 * q[c];
    return;
  }
  double qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  if (qq <= 1e-30) {
    for (int c = 0; c < 3; ++c) X[c] = 2.0 * q[c];
    return;
  }
  double qn = sqrt(qq);
  double hat[3], P = 0.0;
  for (int c = 0; c < 3; ++c) {
    hat[c] = q[c] / qn;
    P = P + (hat[c] * hat[c]) * (hat[c] * hat[c]);
  }
  double ac = 1.0 - delta * (3.0 - 4.0 * P);
  for (int c = 0; c < 3; ++c) {
    double cube = hat[c] * hat[c] * hat[c];
    X[c] = 2.0 * ac * (ac * q[c] + 16.0 * delta * qn * (cube - P * hat[c]));
  }
}

/* Face gradient of one scalar field at the face (i,j,k)->(i,j,k)+e_d: the
 * normal difference, and when full != 0 the two tangential components as the
 * average of the central differences of the two face cells. */
static void face_gradient(const orc_grid* g, const double* f, int i, int j,
                          int k, int d, int full, double gr[3]) {
  int iu = i + UNIT[d][0], ju = j + UNIT[d][1], ku = k + UNIT[d][2];
  double uL = f[cell(g, i, j, k)], uU = f[cell(g, iu, ju, ku)];
  gr[0] = gr[1] = gr[2] = 0.0;
  gr[d] = (uU - uL) / g->dx;
  if (!full) return;
  for (int t = 0; t < 3; ++t) {
    if (t == d) continue;
    double a = at(g, f, i, j, k, t, +1), b = at(g, f, iu, ju, ku, t, +1);
    double c = at(g, f, i, j, k, t, -1), e = at(g, f, iu, ju, ku, t, -1);
    gr[t] = ((a + b) - (c + e)) / (4.0 * g->dx);
  }
}

static int is_boundary_face(const orc_grid* g, int k, int d) {
  return d == 2 && (k < 0 || k >= g->nz - 1);
}

void orc_phi_face(const orc_grid* g, const orc_params* p, const double* phi,
                  int i, int j, int k, int d, double F[4], double S[4]) {
  for (int a = 0; a < NP; ++a) F[a] = S[a] = 0.0;
  if (is_boundary_face(g, k, d)) return;
  const size_t n = ncells(g);
  const int full = anisotropy_active(p);
  double pb[4], gr[4][3];
  int iu = i + UNIT[d][0], ju = j + UNIT[d][1], ku = k + UNIT[d][2];
  for (int a = 0; a < NP; ++a) {
    const double* f = phi + (size_t)a * n;
    pb[a] = 0.5 * (f[cell(g, i, j, k)] + f[cell(g, iu, ju, ku)]);
    face_gradient(g, f, i, j, k, d, full, gr[a]);
  }
  /* normal component of X_ab = dA/dq at q_ab, for a < b */
  double Xd[4][4] = {{0}};
  for (int a = 0; a < NP; ++a)
    for (int b = a + 1; b < NP; ++b) {
      double q[3], X[3];
      for (int c = 0; c < 3; ++c) q[c] = pb[a] * gr[b][c] - pb[b] * gr[a][c];
      orc_aniso_X(q, p->delta[a][b], X);
      Xd[a][b] = X[d];
    }
  /* F_a = sum_{b!=a} gamma_ab (-pb_b) X_ab.e_d   (da/d grad phi_a, normal)
   * S_a = sum_{b!=a} gamma_ab X_ab.e_d (d_d phi_b) (da/dphi_a, face share)
   * with X_ba = -X_ab. */
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) {
      if (b == a) continue;
      double x = a < b ? Xd[a][b] : -Xd[b][a];
      F[a] = F[a] - (p->gamma[a][b] * pb[b]) * x;
      S[a] = S[a] + (p->gamma[a][b] * x) * gr[b][d];
    }
}

void orc_phi_rhs(const orc_grid* g, const orc_params* p, double t,
                 const double* phi, const double* mu, int i, int j, int k,
                 double rhs[4]) {
  const size_t n = ncells(g);
  const size_t c = cell(g, i, j, k);
  const double T = orc_temperature(p, g, (double)k, t);
  double A[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    double Fu[4], Su[4], Fl[4], Sl[4];
    orc_phi_face(g, p, phi, i, j, k, d, Fu, Su);
    orc_phi_face(g, p, phi, i - UNIT[d][0], j - UNIT[d][1], k - UNIT[d][2], d,
                 Fl, Sl);
    for (int a = 0; a < NP; ++a)
      A[a] = A[a] + (0.5 * (Su[a] + Sl[a]) - (Fu[a] - Fl[a]) / g->dx);
  }
  double ph[4], m[2] = {mu[c], mu[n + c]};
  for (int a = 0; a < NP; ++a) ph[a] = phi[(size_t)a * n + c];
  /* driving force dpsi/dphi_a = sum_b psi_b dh_b/dphi_a
   *                          = (2 phi_a / S)(psi_a - sum_b h_b psi_b) */
  double h[4], psi[4], S = 0.0, psibar = 0.0;
  for (int a = 0; a < NP; ++a) S = S + ph[a] * ph[a];
  interp_h(ph, h);
  for (int a = 0; a < NP; ++a) {
    psi[a] = psi_of(p, a, m, T);
    psibar = psibar + h[a] * psi[a];
  }
  const double k16 = 16.0 / (ORC_PI * ORC_PI);
  for (int a = 0; a < NP; ++a) {
    double dpsi = (2.0 * ph[a] / S) * (psi[a] - psibar);
    /* multi-obstacle derivative domega/dphi_a */
    double pair = 0.0, triple = 0.0;
    for (int b = 0; b < NP; ++b)
      if (b != a) pair = pair + p->gamma[a][b] * ph[b];
    for (int b = 0; b < NP; ++b)
      for (int e = b + 1; e < NP; ++e)
        if (b != a && e != a) triple = triple + ph[b] * ph[e];
    double domega = k16 * pair + p->gamma3 * triple;
    rhs[a] = (p->eps * T) * A[a] + (T / p->eps) * domega + dpsi;
  }
}

void orc_phi_cell(const orc_grid* g, const orc_params* p, double t,
                  const double* phi, const double* mu, int i, int j, int k,
                  double out[4]) {
  const size_t n = ncells(g);
  const size_t c = cell(g, i, j, k);
  double rhs[4], y[4];
  orc_phi_rhs(g, p, t, phi, mu, i, j, k, rhs);
  double mean = (((rhs[0] + rhs[1]) + rhs[2]) + rhs[3]) / (double)NP;
  for (int a = 0; a < NP; ++a)
    y[a] = phi[(size_t)a * n + c] -
           p->dt / (p->tau[a] * p->eps) * (rhs[a] - mean);
  orc_project(y, out);
}

/* ---------------------------------------------------------- mu evolution */

void orc_mu_face(const orc_grid* g, const orc_params* p, double t,
                 const double* phi0, const double* phi1, const double* mu,
                 int i, int j, int k, int d, double Phi[2], double J[2]) {
  Phi[0] = Phi[1] = J[0] = J[1] = 0.0;
  if (is_boundary_face(g, k, d)) return;
  const size_t n = ncells(g);
  const double Tf =
      orc_temperature(p, g, d == 2 ? (double)k + 0.5 : (double)k, t);
  int iu = i + UNIT[d][0], ju = j + UNIT[d][1], ku = k + UNIT[d][2];
  const size_t cL = cell(g, i, j, k), cU = cell(g, iu, ju, ku);
  double pb[4], mL[2], mU[2], mb[2];
  for (int a = 0; a < NP; ++a)
    pb[a] = 0.5 * (phi0[(size_t)a * n + cL] + phi0[(size_t)a * n + cU]);
  for (int q = 0; q < NM; ++q) {
    mL[q] = mu[(size_t)q * n + cL];
    mU[q] = mu[(size_t)q * n + cU];
    mb[q] = 0.5 * (mL[q] + mU[q]);
  }
  /* diffusive flux M_i d_d mu_i with M_i = sum_a D_a phi_a chi_ai(T_f) */
  double diff[2];
  for (int q = 0; q < NM; ++q) {
    double M = 0.0;
    for (int a = 0; a < NP; ++a)
      M = M + (p->D[a] * pb[a]) * chi_of(p, a, q, Tf);
    diff[q] = M * (mU[q] - mL[q]) / g->dx;
  }
  if (p->antitrapping) {
    /* Eq. (4), normal component on this face:
     * J_i = (pi eps/4) sum_{a != l} [g_a h_l / sqrt(phi_a phi_l)] dphi_a/dt
     *       (n_a . n_l) (c^l_i - c^a_i) (n_a . e_d)
     * with g_a h_l / sqrt(phi_a phi_l) = sqrt(phi_a phi_l) phi_l / S. */
    double gr[4][3], nv[4][3];
    for (int a = 0; a < NP; ++a) {
      face_gradient(g, phi0 + (size_t)a * n, i, j, k, d, 1, gr[a]);
      double nrm = sqrt(gr[a][0] * gr[a][0] + gr[a][1] * gr[a][1] +
                        gr[a][2] * gr[a][2]);
      for (int c = 0; c < 3; ++c) nv[a][c] = nrm > 0.0 ? gr[a][c] / nrm : 0.0;
    }
    double Sb = pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2] + pb[3] * pb[3];
    for (int a = 0; a < LQ; ++a) {
      double prod = pb[a] * pb[LQ];
      double w = prod > 0.0 ? sqrt(prod) * pb[LQ] / Sb : 0.0;
      double rate = 0.5 *
                    ((phi1[(size_t)a * n + cL] - phi0[(size_t)a * n + cL]) +
                     (phi1[(size_t)a * n + cU] - phi0[(size_t)a * n + cU])) /
                    p->dt;
      double nn = nv[a][0] * nv[LQ][0] + nv[a][1] * nv[LQ][1] +
                  nv[a][2] * nv[LQ][2];
      double coef = w * rate * nn * nv[a][d];
      for (int q = 0; q < NM; ++q) {
        double dc = conc_of(p, LQ, q, mb, Tf) - conc_of(p, a, q, mb, Tf);
        J[q] = J[q] + coef * dc;
      }
    }
    const double pre = ORC_PI * p->eps / 4.0;
    for (int q = 0; q < NM; ++q) J[q] = pre * J[q];
  }
  for (int q = 0; q < NM; ++q) Phi[q] = diff[q] - J[q];
}

void orc_mu_cell(const orc_grid* g, const orc_params* p, double t0, double t1,
                 const double* phi0, const double* phi1, const double* mu,
                 int i, int j, int k, double out[2]) {
  const size_t n = ncells(g);
  const size_t c = cell(g, i, j, k);
  double m[2] = {mu[c], mu[n + c]};
  if (p->mu_frozen) {
    out[0] = m[0];
    out[1] = m[1];
    return;
  }
  double div[2] = {0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    double Pu[2], Pl[2], Ju[2], Jl[2];
    orc_mu_face(g, p, t0, phi0, phi1, mu, i, j, k, d, Pu, Ju);
    orc_mu_face(g, p, t0, phi0, phi1, mu, i - UNIT[d][0], j - UNIT[d][1],
                k - UNIT[d][2], d, Pl, Jl);
    for (int q = 0; q < NM; ++q) div[q] = div[q] + (Pu[q] - Pl[q]) / g->dx;
  }
  const double Tn = orc_temperature(p, g, (double)k, t0);
  const double Tn1 = orc_temperature(p, g, (double)k, t1);
  double p0[4], p1[4], h0[4], h1[4];
  for (int a = 0; a < NP; ++a) {
    p0[a] = phi0[(size_t)a * n + c];
    p1[a] = phi1[(size_t)a * n + c];
  }
  interp_h(p0, h0);
  interp_h(p1, h1);
  for (int q = 0; q < NM; ++q) {
    /* c(phi,mu,T) = sum_a h_a c_a(mu,T).  Split c^{n+1} - c^n into
     * chi(phi^{n+1},T^{n+1}) (mu^{n+1} - mu^n) + src, so that
     * c^{n+1} - c^n = dt div(M grad mu - J_at) holds exactly. */
    const double cref = cbar_of(p, LQ, q, Tn);
    double src = 0.0, chi = 0.0;
    for (int a = 0; a < NP; ++a) {
      double dchi = chi_of(p, a, q, Tn1) - chi_of(p, a, q, Tn);
      double dcb = cbar_of(p, a, q, Tn1) - cbar_of(p, a, q, Tn);
      src = src + ((h1[a] - h0[a]) * (conc_of(p, a, q, m, Tn) - cref) +
                   h1[a] * (dchi * m[q] + dcb));
      chi = chi + h1[a] * chi_of(p, a, q, Tn1);
    }
    out[q] = m[q] + (p->dt * div[q] - src) / chi;
  }
}

/* ------------------------------------------------------------ sweeps */

void orc_phi_sweep(const orc_grid* g, const orc_params* p, double t,
                   const double* phi, const double* mu, double* phi_out,
                   int nthreads) {
  const size_t n = ncells(g);
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        double out[4];
        orc_phi_cell(g, p, t, phi, mu, i, j, k, out);
        size_t c = cell(g, i, j, k);
        for (int a = 0; a < NP; ++a) phi_out[(size_t)a * n + c] = out[a];
      }
}

void orc_mu_sweep(const orc_grid* g, const orc_params* p, double t0, double t1,
                  const double* phi0, const double* phi1, const double* mu,
                  double* mu_out, int nthreads) {
  const size_t n = ncells(g);
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        double out[2];
        orc_mu_cell(g, p, t0, t1, phi0, phi1, mu, i, j, k, out);
        size_t c = cell(g, i, j, k);
        for (int q = 0; q < NM; ++q) mu_out[(size_t)q * n + c] = out[q];
      }
}

static void set_ghost_plane(const orc_grid* ge, const orc_params* p, double* phi,
                            double* mu) {
  const size_t plane = (size_t)ge->nx * ge->ny, n = ncells(ge);
  const size_t top = plane * (size_t)(ge->nz - 1);
  for (size_t c = 0; c < plane; ++c) {
    for (int a = 0; a < NP; ++a) phi[(size_t)a * n + top + c] = a == ORC_LIQ ? 1.0 : 0.0;
    if (mu)
      for (int q = 0; q < NM; ++q) mu[(size_t)q * n + top + c] = p->mu_top[q];
  }
}

/* Dirichlet top: copy the fields into a grid one plane taller whose top
 * plane is the ghost, step there, copy planes 0..nz-1 back. */
static int run_dirichlet(const orc_grid* g, const orc_params* p, int64_t step0,
                         int64_t nsteps, double* phi, double* mu, int nthreads) {
  orc_grid ge = *g;
  ge.nz = g->nz + 1;
  const size_t n = ncells(g), ne = ncells(&ge);
  double* pe = (double*)malloc(sizeof(double) * NP * ne);
  double* me = (double*)malloc(sizeof(double) * NM * ne);
  double* pe2 = (double*)malloc(sizeof(double) * NP * ne);
  double* me2 = (double*)malloc(sizeof(double) * NM * ne);
  if (!pe || !me || !pe2 || !me2) {
    free(pe);
    free(me);
    free(pe2);
    free(me2);
    return -1;
  }
  for (int a = 0; a < NP; ++a) memcpy(pe + (size_t)a * ne, phi + (size_t)a * n, sizeof(double) * n);
  for (int q = 0; q < NM; ++q) memcpy(me + (size_t)q * ne, mu + (size_t)q * n, sizeof(double) * n);
  for (int64_t s = step0; s < step0 + nsteps; ++s) {
    double t0 = (double)s * p->dt, t1 = (double)(s + 1) * p->dt;
    set_ghost_plane(&ge, p, pe, me);
    orc_phi_sweep(&ge, p, t0, pe, me, pe2, nthreads);
    set_ghost_plane(&ge, p, pe2, NULL);
    orc_mu_sweep(&ge, p, t0, t1, pe, pe2, me, me2, nthreads);
    memcpy(pe, pe2, sizeof(double) * NP * ne);
    memcpy(me, me2, sizeof(double) * NM * ne);
  }
  for (int a = 0; a < NP; ++a) memcpy(phi + (size_t)a * n, pe + (size_t)a * ne, sizeof(double) * n);
  for (int q = 0; q < NM; ++q) memcpy(mu + (size_t)q * n, me + (size_t)q * ne, sizeof(double) * n);
  free(pe);
  free(me);
  free(pe2);
  free(me2);
  return 0;
}

int orc_run(const orc_grid* g, const orc_params* p, int64_t step0,
            int64_t nsteps, double* phi, double* mu, int nthreads) {
  if (p->top_dirichlet) return run_dirichlet(g, p, step0, nsteps, phi, mu, nthreads);
  const size_t n = ncells(g);
  double* phi2 = (double*)malloc(sizeof(double) * NP * n);
  double* mu2 = (double*)malloc(sizeof(double) * NM * n);
  if (!phi2 || !mu2) {
    free(phi2);
    free(mu2);
    return -1;
  }
  /* Algorithm 1: phi_dst <- phi-kernel(phi_src, mu_src);
   *              mu_dst  <- mu-kernel(mu_src, phi_src, phi_dst); swap.
   * Times are products t_n = n dt, never accumulated. */
  for (int64_t s = step0; s < step0 + nsteps; ++s) {
    double t0 = (double)s * p->dt, t1 = (double)(s + 1) * p->dt;
    orc_phi_sweep(g, p, t0, phi, mu, phi2, nthreads);
    orc_mu_sweep(g, p, t0, t1, phi, phi2, mu, mu2, nthreads);
    memcpy(phi, phi2, sizeof(double) * NP * n);
    memcpy(mu, mu2, sizeof(double) * NM * n);
  }
  free(phi2);
  free(mu2);
  return 0;
}

/* ------------------------------------------------------ moving window */

int orc_window_shift(const orc_grid* g, int32_t zw, const double mu_fill[2],
                     double* phi, double* mu) {
  const size_t plane = (size_t)g->nx * g->ny, n = ncells(g);
  const double* pl = phi + (size_t)ORC_LIQ * n + (size_t)zw * plane;
  double sum = 0.0;
  for (size_t c = 0; c < plane; ++c) sum += pl[c];
  if (!(sum < 0.5 * (double)plane)) return 0;
  for (int a = 0; a < NP; ++a) {
    double* f = phi + (size_t)a * n;
    memmove(f, f + plane, sizeof(double) * plane * (size_t)(g->nz - 1));
    double* top = f + plane * (size_t)(g->nz - 1);
    for (size_t c = 0; c < plane; ++c) top[c] = a == ORC_LIQ ? 1.0 : 0.0;
  }
  for (int q = 0; q < NM; ++q) {
    double* f = mu + (size_t)q * n;
    memmove(f, f + plane, sizeof(double) * plane * (size_t)(g->nz - 1));
    double* top = f + plane * (size_t)(g->nz - 1);
    for (size_t c = 0; c < plane; ++c) top[c] = mu_fill[q];
  }
  return 1;
}

int orc_run_window(const orc_grid* g, const orc_params* p, int64_t step0,
                   int64_t nsteps, int32_t zw, const double mu_fill[2],
                   int64_t* shifts, double* phi, double* mu, int nthreads) {
  orc_params q = *p;
  for (int64_t s = step0; s < step0 + nsteps; ++s) {
    if (zw > 0) *shifts += orc_window_shift(g, zw, mu_fill, phi, mu);
    q.zoff = p->zoff + (double)(*shifts) * g->dx;
    if (orc_run(g, &q, s, 1, phi, mu, nthreads) != 0) return -1;
  }
  return 0;
}

/* ------------------------------------------------------ initial state */

void orc_init_voronoi(const orc_grid* g, uint64_t seed, int32_t nseeds,
                      int32_t solid_height, const double mu_init[2],
                      double* phi, double* mu) {
  const size_t n = ncells(g);
  double* sx = (double*)malloc(sizeof(double) * (size_t)(nseeds > 0 ? nseeds : 1));
  double* sy = (double*)malloc(sizeof(double) * (size_t)(nseeds > 0 ? nseeds : 1));
  uint64_t st = seed;
  for (int s = 0; s < nseeds; ++s) {
    sx[s] = (double)(orc_splitmix64_next(&st) >> 11) * 0x1.0p-53 * g->nx;
    sy[s] = (double)(orc_splitmix64_next(&st) >> 11) * 0x1.0p-53 * g->ny;
  }
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      /* nearest seed by periodic minimum-image distance; lowest index wins */
      int best = 0;
      double bd = INFINITY;
      double cx = (double)i + 0.5, cy = (double)j + 0.5;
      for (int s = 0; s < nseeds; ++s) {
        double ddx = fabs(cx - sx[s]), ddy = fabs(cy - sy[s]);
        if (g->nx - ddx < ddx) ddx = g->nx - ddx;
        if (g->ny - ddy < ddy) ddy = g->ny - ddy;
        double d2 = ddx * ddx + ddy * ddy;
        if (d2 < bd) {
          bd = d2;
          best = s;
        }
      }
      int solid_phase = best % 3;
      for (int k = 0; k < g->nz; ++k) {
        size_t c = cell(g, i, j, k);
        int ph = (k < solid_height && nseeds > 0) ? solid_phase : LQ;
        for (int a = 0; a < NP; ++a) phi[(size_t)a * n + c] = a == ph ? 1.0 : 0.0;
        for (int q = 0; q < NM; ++q) mu[(size_t)q * n + c] = mu_init[q];
      }
    }
  free(sx);
  free(sy);
}

/* ------------------------------------------------------- diagnostics */

void orc_diagnostics(const orc_grid* g, const orc_params* p, double t,
                     const double* phi, const double* mu, orc_diag* out) {
  const size_t n = ncells(g);
  memset(out, 0, sizeof(*out));
  out->phi_min = INFINITY;
  out->phi_max = -INFINITY;
  for (int k = 0; k < g->nz; ++k) {
    const double T = orc_temperature(p, g, (double)k, t);
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        size_t c = cell(g, i, j, k);
        double ph[4], h[4], m[2] = {mu[c], mu[n + c]}, s = 0.0;
        int bad = 0;
        for (int a = 0; a < NP; ++a) {
          ph[a] = phi[(size_t)a * n + c];
          if (!isfinite(ph[a])) bad = 1;
          out->sum_phi[a] += ph[a];
          s = s + ph[a];
          if (ph[a] < out->phi_min) out->phi_min = ph[a];
          if (ph[a] > out->phi_max) out->phi_max = ph[a];
        }
        for (int q = 0; q < NM; ++q)
          if (!isfinite(m[q])) bad = 1;
        out->nonfinite += bad;
        double dev = fabs(s - 1.0);
        if (dev > out->max_simplex_dev) out->max_simplex_dev = dev;
        interp_h(ph, h);
        for (int q = 0; q < NM; ++q) {
          double cq = 0.0;
          for (int a = 0; a < NP; ++a) cq = cq + h[a] * conc_of(p, a, q, m, T);
          out->sum_c[q] += cq;
        }
      }
  }
}
