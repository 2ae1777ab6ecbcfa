/*
 * pf_oracle.h -- plain FP64 CPU oracle of the grand-potential multi-phase-field
 * time step (Bauer et al., "Massively Parallel Phase-Field Simulations for
 * Ternary Eutectic Directional Solidification", SC'15, arXiv:1506.01684).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * Fields are unpadded, x fastest: phi[a][z][y][x] (a = 0..3, phase 3 = liquid),
 * mu[i][z][y][x] (i = 0..1).  Everything is FP64, compiled without FMA
 * contraction (-ffp-contract=off) so every expression rounds as written.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NPHASE 4
#define ORC_NMU 2
#define ORC_LIQ 3

typedef struct {
  int32_t nx, ny, nz;
  double dx;
} orc_grid;

typedef struct {
  double eps;              /* interface width parameter epsilon        */
  double tau[4];           /* relaxation parameters tau_alpha          */
  double gamma[4][4];      /* pair surface energies (symmetric)        */
  double gamma3;           /* uniform triple-junction coefficient      */
  double delta[4][4];      /* cubic anisotropy strength per pair       */
  double chi0[4][2], chi1[4][2]; /* susceptibility chi = chi0+chi1(T-TE) */
  double c0[4][2], c1[4][2];     /* offsets cbar = c0 + c1 (T-TE)        */
  double w0[4], w1[4];           /* omega_bar = w0 + w1 (T-TE)           */
  double D[4];             /* diffusivities                            */
  double TE, T0, G, v, zoff; /* T(z,t) = T0 + G (z + zoff - v t)      */
  double dt;
  int32_t antitrapping;    /* 1: include the anti-trapping current      */
  int32_t mu_frozen;       /* 1: mu is not evolved (tests only)        */
  int32_t top_dirichlet;   /* 1: Dirichlet top (ghost plane above the top
                            * is liquid, phi = e_liquid, at mu = mu_top);
                            * 0: zero-flux mirror, as at the bottom      */
  int32_t pad;
  double mu_top[2];
} orc_params;

typedef struct {
  double sum_c[2];
  double sum_phi[4];
  double max_simplex_dev;
  double phi_min, phi_max;
  int64_t nonfinite;
} orc_diag;

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): advance *state, return output. */
uint64_t orc_splitmix64_next(uint64_t* state);

/* Frozen temperature T(zc, t) = T0 + G (zc dx + zoff - v t); zc in cell units. */
double orc_temperature(const orc_params* p, const orc_grid* g, double zc, double t);

/* Explicit stability bound min(dt_phi, dt_mu) at t = 0 (the default dt is a
 * quarter of it). */
double orc_stability_bound(const orc_params* p, const orc_grid* g);

/* Euclidean projection of y onto the Gibbs simplex, then renormalisation. */
void orc_project(const double y[4], double x[4]);

/* Derivative X = d(ac(q)^2 |q|^2)/dq of the (cubic-anisotropic) pair gradient
 * energy at the generalised gradient vector q. */
void orc_aniso_X(const double q[3], double delta, double X[3]);

/* phi face (i,j,k) -> (i,j,k)+e_d: normal flux F_a and face share S_a of
 * d a / d phi_a.  Faces on the z boundaries (k < 0 or k >= nz-1 for d = 2)
 * carry zero flux. */
void orc_phi_face(const orc_grid* g, const orc_params* p, const double* phi,
                  int i, int j, int k, int d, double F[4], double S[4]);

/* Right-hand side rhs_a of the phi equation at cell (i,j,k), before the
 * Lagrange mean is subtracted. */
void orc_phi_rhs(const orc_grid* g, const orc_params* p, double t,
                 const double* phi, const double* mu, int i, int j, int k,
                 double rhs[4]);

/* New phi of one cell (explicit Euler + projection). */
void orc_phi_cell(const orc_grid* g, const orc_params* p, double t,
                  const double* phi, const double* mu, int i, int j, int k,
                  double out[4]);

/* mu face flux Phi_i = M_i d mu_i - J_i and the anti-trapping part J_i. */
void orc_mu_face(const orc_grid* g, const orc_params* p, double t,
                 const double* phi0, const double* phi1, const double* mu,
                 int i, int j, int k, int d, double Phi[2], double J[2]);

/* New mu of one cell. t0 = n dt, t1 = (n+1) dt. */
void orc_mu_cell(const orc_grid* g, const orc_params* p, double t0, double t1,
                 const double* phi0, const double* phi1, const double* mu,
                 int i, int j, int k, double out[2]);

/* Whole-domain sweeps (z planes split over nthreads; bitwise independent of
 * the thread count because every cell reads only source arrays). */
void orc_phi_sweep(const orc_grid* g, const orc_params* p, double t,
                   const double* phi, const double* mu, double* phi_out,
                   int nthreads);
void orc_mu_sweep(const orc_grid* g, const orc_params* p, double t0, double t1,
                  const double* phi0, const double* phi1, const double* mu,
                  double* mu_out, int nthreads);

/* nsteps full time steps starting at step index step0, in place.  With a
 * Dirichlet top the sweeps run on the grid extended by the ghost plane
 * (index nz, held at its fixed values before each sweep), so the face
 * between the top plane and the ghost is evaluated like any interior face;
 * only planes 0..nz-1 are kept. */
int orc_run(const orc_grid* g, const orc_params* p, int64_t step0,
            int64_t nsteps, double* phi, double* mu, int nthreads);

/* Moving window (Sec. 3.3; the technique of Vondrous et al. 2014 that the
 * paper cites): the window follows the solidification front along z.  If
 * the mean liquid fraction of plane zw (sum over the plane of phi_liquid,
 * in FP64, x fastest, compared with nx ny / 2) is below one half, the front
 * has passed zw: every plane moves down by one (the bottom plane, deep in
 * the solid whose evolution the paper neglects, is dropped), the top plane
 * becomes liquid (phi = e_liquid) at mu = mu_fill, and 1 is returned (the
 * caller then counts one more shift, i.e. adds dx to zoff).  Otherwise the
 * fields are untouched and 0 is returned. */
int orc_window_shift(const orc_grid* g, int32_t zw, const double mu_fill[2],
                     double* phi, double* mu);

/* orc_run with a moving window at plane zw (> 0): before each step the
 * window is checked and shifted as above; shifts counts the shifts made so
 * far (in and out), and the temperature of step s uses
 * zoff + shifts dx. */
int orc_run_window(const orc_grid* g, const orc_params* p, int64_t step0,
                   int64_t nsteps, int32_t zw, const double mu_fill[2],
                   int64_t* shifts, double* phi, double* mu, int nthreads);

/* Voronoi-seeded initial state: solid lamellae below solid_height, liquid
 * above, mu = mu_init everywhere. */
void orc_init_voronoi(const orc_grid* g, uint64_t seed, int32_t nseeds,
                      int32_t solid_height, const double mu_init[2],
                      double* phi, double* mu);

/* Diagnostics at time t: total concentration, phase sums, simplex deviation,
 * phi range and count of non-finite values. */
void orc_diagnostics(const orc_grid* g, const orc_params* p, double t,
                     const double* phi, const double* mu, orc_diag* out);

/* Interface mesh of phase `phase` (output path, Sec. 3.2): marching cubes
 * over the cell-centre grid for phi_phase = iso, reading and rules at the
 * top of pf_oracle_mesh.c.  Writes up to `capacity` triangles (9 floats
 * each: three vertices xyz, cell-index units) in cube order (x fastest,
 * then y, z) and returns the total count. */
int64_t orc_mesh_phase(const orc_grid* g, const double* phi, int32_t phase, double iso,
                       float* out, int64_t capacity);

#ifdef __cplusplus
}
#endif
#endif
