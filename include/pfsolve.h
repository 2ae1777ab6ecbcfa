/*
 * pfsolve.h -- C ABI of the MI355X phase-field stepper.
 *
 * The library advances the grand-potential multi-phase-field model of
 * Bauer et al., "Massively Parallel Phase-Field Simulations for Ternary
 * Eutectic Directional Solidification" (SC'15, arXiv:1506.01684): N = 4
 * order parameters phi (three solids, index 0..2, and the liquid, index 3)
 * on the Gibbs simplex and K-1 = 2 chemical potentials mu on a regular 3D
 * grid of equidistant cells (Sec. 2), with explicit Euler time steps made of
 * a phi-sweep (Eqs. (1)-(2)) followed by a mu-sweep (Eqs. (3)-(4)) that reads
 * mu_src, phi_src and phi_dst, then a swap of source and destination fields
 * (Algorithm 1).  Temperature is frozen: T(z,t) = T0 + G (z + zoff - v t)
 * (Sec. 2 and Sec. 3.3).  Boundaries: periodic in x and y, zero-flux mirror
 * in z.  The initial state is solid Voronoi nuclei below a liquid (Sec. 2.1).
 *
 * Conventions shared by every call:
 *  - No exception crosses the ABI; every fallible call returns pf_status and
 *    on failure stores a message readable with pf_last_error() (per thread).
 *  - Host arrays are always owned by the caller and copied in or out; host
 *    field arrays are FP64, unpadded, x fastest: phi[a][z][y][x] (a = 0..3),
 *    mu[i][z][y][x] (i = 0..1).
 *  - Device memory is owned by the library unless the caller lends a buffer
 *    (pf_device_buffer); a lent buffer must outlive the domain.
 *  - Work is enqueued on the HIP stream given at creation (NULL = the null
 *    stream) and is asynchronous unless a call says it synchronises.
 *  - Calls on different domains may run concurrently from different threads;
 *    a single domain or pack is not re-entrant.
 */
#ifndef PFSOLVE_H
#define PFSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_domain pf_domain; /* opaque: one grid and its fields */
typedef struct pf_pack pf_pack;     /* opaque: many domains stepped together */

typedef enum {
  PF_OK = 0,
  PF_ERR_INVALID_ARG = 1, /* a size, pointer or parameter is out of range */
  PF_ERR_STATE = 2,       /* call made in the wrong order                 */
  PF_ERR_UNSTABLE = 3,    /* explicit dt above the stability bound        */
  PF_ERR_OOM = 4,         /* device allocation failed / buffer too small  */
  PF_ERR_DEVICE = 5,      /* a HIP runtime call failed                    */
  PF_ERR_NONFINITE = 6,   /* diagnostics found NaN or Inf in the fields   */
  PF_ERR_IO = 7           /* a file could not be opened, read or written  */
} pf_status;

/* Storage and arithmetic precision of a domain.  PF_FP32 stores fields and
 * evaluates the sweeps in FP32 with FP32 accumulation, but keeps the
 * temperature, time, per-plane coefficients, the simplex projection and the
 * diagnostic sums in FP64. */
typedef enum { PF_FP64 = 0, PF_FP32 = 1 } pf_precision;

typedef struct {
  int32_t nx, ny, nz; /* cells per axis, each >= 1                         */
  int32_t prec;       /* pf_precision                                      */
  double dx;          /* cell spacing (> 0), the same on every axis (Sec. 2) */
} pf_domain_desc;

typedef struct {
  void* base;   /* device pointer, 256-byte aligned                       */
  size_t bytes; /* at least pf_required_bytes()                           */
} pf_device_buffer;

/* Model parameters (all FP64 on the host; copied by pf_set_params).
 * Functional forms (the paper names the terms of Eqs. (1)-(4) but not their
 * forms; these are the forms implemented):
 *   gradient energy a = sum_{a<b} gamma_ab ac(q_ab)^2 |q_ab|^2,
 *     q_ab = phi_a grad phi_b - phi_b grad phi_a,
 *     ac(q) = 1 - delta_ab (3 - 4 sum_i (q_i/|q|)^4)   (cubic; 0 <= delta < 1/15)
 *   obstacle omega = 16/pi^2 sum_{a<b} gamma_ab phi_a phi_b
 *                    + gamma3 sum_{a<b<c} phi_a phi_b phi_c
 *   grand potentials psi_a = -1/2 sum_i chi_ai(T) mu_i^2 - sum_i cbar_ai(T) mu_i
 *                    + wbar_a(T), with chi = chi0 + chi1 (T-TE),
 *                    cbar = c0 + c1 (T-TE), wbar = w0 + w1 (T-TE)
 *   interpolation h_a = phi_a^2 / sum_b phi_b^2; mobility sum_a D_a phi_a chi_ai */
typedef struct {
  double eps;             /* interface width parameter (> 0)               */
  double tau[4];          /* relaxation parameters (> 0)                   */
  double gamma[4][4];     /* pair coefficients, symmetric, >= 0            */
  double gamma3;          /* uniform triple coefficient (>= 0)             */
  double aniso_delta[4][4]; /* cubic anisotropy per pair, symmetric        */
  double chi0[4][2], chi1[4][2]; /* susceptibility coefficients            */
  double c0[4][2], c1[4][2];     /* concentration offsets                  */
  double w0[4], w1[4];           /* grand-potential offsets                */
  double D[4];                   /* diffusivities (>= 0)                   */
  double TE, T0, G, v, zoff;     /* T(z,t) = T0 + G (z + zoff - v t)       */
  double dt;          /* <= 0: a quarter of the stability bound            */
  int32_t antitrapping; /* 1: include the anti-trapping current of Eq. (4) */
  int32_t mu_frozen;    /* 1: mu is held fixed (for tests of the phi part) */
  int32_t diag_every;   /* run diagnostics every n steps inside pf_step (0 = never) */
  int32_t shortcuts;    /* 1: skip work whose result is exactly known (Sec. 3.3
                         * shortcuts, made exact): phi faces whose normal
                         * differences all vanish carry exactly zero flux, and
                         * a pure cell with zero face sums that is a fixed
                         * point of its plane keeps its value.  Results are
                         * bitwise identical to 0 (evaluate everything). */
  int32_t window_z;     /* moving window along z (Sec. 3.3, the technique of
                         * Vondrous et al. 2014 the paper cites): 0 = off, else
                         * a plane index in [1, nz-2].  Before each step, if the
                         * mean liquid fraction of plane window_z (FP64 sum of
                         * phi_3 over the plane) is below 1/2, the front has
                         * passed it: every plane moves down by one (plane 0,
                         * deep in the solid, is dropped), the top plane becomes
                         * liquid (phi = e_3) at mu = mu_fill, and the origin of
                         * z moves up by dx (the temperature uses
                         * zoff + shifts dx).  At most one shift per step. */
  int32_t top_bc;       /* top boundary (Sec. 3.1 boundary handling): 0 =
                         * zero-flux mirror, as at the bottom; 1 = Dirichlet:
                         * a ghost plane above the top plane is held at
                         * liquid (phi = e_3) at mu = mu_fill, and the face to
                         * it is evaluated like any interior face */
  double mu_fill[2];    /* mu of the liquid a window shift adds and of the
                         * Dirichlet ghost plane */
} pf_params;

typedef enum { PF_INIT_VORONOI = 0, PF_INIT_HOST = 1 } pf_init_kind;

typedef struct {
  int32_t kind;         /* pf_init_kind                                    */
  int32_t nseeds;       /* VORONOI: number of 2D seeds (>= 0)              */
  uint64_t seed;        /* VORONOI: SplitMix64 seed for seed positions     */
  int32_t solid_height; /* VORONOI: cells with z < solid_height are solid  */
  int32_t reserved;
  double mu_init[2];    /* VORONOI: uniform initial mu                     */
  const double* phi;    /* HOST: 4*nx*ny*nz values, layout as above        */
  const double* mu;     /* HOST: 2*nx*ny*nz values                         */
} pf_init;

typedef struct {
  double t;               /* time of the state the diagnostics describe   */
  int64_t step;           /* its step index                               */
  double sum_c[2];        /* sum over cells of c_i = sum_a h_a c_ai(mu,T) */
  double sum_phi[4];      /* sum over cells of each phi_a                 */
  double max_simplex_dev; /* max over cells of |sum_a phi_a - 1|           */
  double phi_min, phi_max;
  int64_t nonfinite;      /* cells holding a NaN or Inf in any field      */
  int64_t window_shifts;  /* moving-window shifts since pf_init_fields    */
  int32_t light_items;    /* work items of the last step whose faces cannot
                           * carry the anti-trapping current (Eq. 4: no
                           * liquid, or only liquid, around them), counted
                           * by the FP64 tiled sweep; 0 in FP32, with the
                           * direct variant, with the shortcuts off, and
                           * before the first step                         */
  int32_t work_items;     /* work items per sweep of this domain (x-y
                           * tiles times z chunks)                        */
  int32_t fixed_items;    /* work items of the last step whose phi the
                           * tiled sweep copied unchanged: every cell in and
                           * around them held one pure phase that its planes
                           * mark as a fixed point (Sec. 3.3 bulk shortcut,
                           * exact); 0 with the shortcuts off, the direct
                           * variant, and before the first step           */
  int32_t mu_pure_items;  /* work items of the last step whose mu the tiled
                           * sweep evaluated from mu alone: they and every
                           * cell their stencils read held one pure phase
                           * before and after the phi-sweep, so phi^n =
                           * phi^{n+1} = e_a there (Sec. 3.3 bulk shortcut,
                           * exact); 0 with the shortcuts off, mu frozen,
                           * the direct variant, and before the first step */
  int32_t copied_items;   /* of the fixed_items, those whose phi the sweep
                           * had to copy into the copy it writes (the others
                           * were kept in both copies the step before) */
  int32_t reserved;       /* 0 */
} pf_diag;

/* Device bytes a domain needs (both field copies, each with one extra
 * plane per field for the Dirichlet ghost, plus scratch).  Not in the
 * paper: the memory budget of the serving loop (admission against HBM)
 * needs it.  The two copies are Algorithm 1's source and destination
 * fields; the layout is structure of arrays, x fastest, rows padded to
 * 128 bytes.  INVALID_ARG for sizes <= 0, a field plane of 4 GiB or more
 * (padded row bytes times ny: the sweeps address a plane with 32-bit byte
 * offsets) or a total that overflows. */
pf_status pf_required_bytes(const pf_domain_desc* desc, size_t* out);

/* Create a domain on the current HIP device: the regular grid of
 * equidistant cells of Sec. 2 (Sec. 3.1, block structure, with one block
 * per domain here).  Not in the paper as a call: the library's own
 * lifetime management.  borrowed: NULL = allocate, else a caller-owned
 * device buffer of at least pf_required_bytes() that must outlive the
 * domain.  stream: a hipStream_t (NULL = null stream).  Errors:
 * INVALID_ARG for sizes that pf_required_bytes rejects, OOM, DEVICE. */
pf_status pf_create_domain(const pf_domain_desc* desc,
                           const pf_device_buffer* borrowed, void* stream,
                           pf_domain** out);

/* Copy and validate parameters; resolve dt (the model parameters of
 * Sec. 2 and the explicit Euler step of Algorithm 1).  Errors: STATE for a
 * pack member (its descriptor belongs to the pack's captured step);
 * INVALID_ARG for
 * non-positive eps/tau/dx, chi <= 0 over the domain's temperature range,
 * negative gamma or D, delta outside [0, 1/15); UNSTABLE for an explicit dt
 * above the stability bound min(dt_phi, dt_mu) with
 * dt_phi = dx^2 min(tau) / (12 max(gamma) T_max (1+dmax)(1+15 dmax)) and
 * dt_mu = dx^2 min(chi) / (6 max(D chi)). */
pf_status pf_set_params(pf_domain* d, const pf_params* p);

/* The resolved time step and the stability bound. */
pf_status pf_get_dt(const pf_domain* d, double* dt, double* bound);

/* Initialise both sweeps' source fields; resets the step index and the
 * window shift count to 0.  STATE for a pack member.
 * VORONOI (Sec. 2.1): nseeds points drawn with SplitMix64 (Steele, Lea,
 * Flood 2014) as (u nx, u ny), u = (next >> 11) 2^-53, x first; seed s gets
 * solid phase s mod 3; each column takes the nearest seed by periodic
 * minimum-image distance from its centre (i+1/2, j+1/2), lowest index on
 * ties; z < solid_height is solid, the rest liquid; mu = mu_init.
 * HOST: copy (and for FP32 round) the caller's arrays, phi[4][nz][ny][nx]
 * and mu[2][nz][ny][nx] (host memory, read only, still owned by the
 * caller); each field passes through the domain's second field copy on the
 * device, so no memory is allocated.  Synchronises.  Errors: INVALID_ARG
 * (unknown kind, nseeds or solid_height < 0, null HOST arrays) leaves the
 * domain as it was; DEVICE leaves it without fields (step and read calls
 * return STATE until it is initialised again). */
pf_status pf_init_fields(pf_domain* d, const pf_init* init);

/* Resume from a checkpoint (Sec. 3.2 checkpointing): the next step is
 * number `step`, t = step dt (times are products, as the frozen
 * temperature of Sec. 2 is a function of t).  STATE before the fields are
 * set or for a pack member; INVALID_ARG for step < 0.
 * The window shift count is kept; a caller resuming a windowed run from
 * host fields sets pf_params.zoff to the old zoff plus shifts * dx. */
pf_status pf_set_time(pf_domain* d, int64_t step);

/* Enqueue n time steps (Algorithm 1), asynchronously.  Errors: STATE when
 * params or fields are missing; a pending NONFINITE from in-loop
 * diagnostics is reported here or by pf_sync. */
pf_status pf_step(pf_domain* d, int64_t n);

/* As pf_step, and add the device time of each sweep, measured with HIP
 * events on the domain's stream, to *phi_ms and *mu_ms (per-sweep totals
 * over the n steps).  Synchronises at the end. */
pf_status pf_step_timed(pf_domain* d, int64_t n, double* phi_ms,
                        double* mu_ms);

/* Wait for all enqueued work; report asynchronous errors.  Not in the
 * paper: the stream model of this library (every call enqueues on the
 * domain's HIP stream).  Reports NONFINITE when in-loop diagnostics found
 * a non-finite cell, DEVICE for a HIP error. */
pf_status pf_sync(pf_domain* d);

/* Copy the current state to host (FP32 widened to FP64) and/or compute the
 * diagnostics of the current state; any pointer may be NULL.  phi and mu
 * are caller-owned host arrays of 4 and 2 times nx ny nz doubles, laid out
 * as for pf_init_fields.  Each field is packed on the device into the
 * copy that does not hold the state (no memory is allocated); the state is
 * unchanged, and the next step's bulk shortcut copies the chunks it would
 * otherwise have found in both copies.  Synchronises.  Returns NONFINITE
 * (after filling the outputs) if the diagnostics count any non-finite
 * cell. */
pf_status pf_read_fields(pf_domain* d, double* phi, double* mu, pf_diag* diag);

/* Number of completed steps of the current state: the time level n of
 * Algorithm 1's source fields (t = n dt).  Synchronises with the device's
 * step counter. */
pf_status pf_get_step(const pf_domain* d, int64_t* step);

/* Synchronise and free owned memory (a borrowed buffer is left to its
 * owner); a pack member is removed from its pack first.  NULL is accepted.
 * Not in the paper: the library's own lifetime management. */
void pf_destroy(pf_domain* d);

/* ------------------------------------------------------------ output path
 * Sec. 3.2 (Input/Output): the arithmetic is FP64, checkpoints hold the
 * state in single precision, and results are written as triangle meshes of
 * the interfaces, one per phase, from a marching-cubes pass over phi.  None
 * of these calls is part of the time step.
 *
 * Checkpoint file, little endian: a 64-byte header
 *   char magic[8] = "PFCKPT01"; int32 nx, ny, nz; int32 prec (of the domain
 *   that wrote it); int64 step; int64 window_shifts; double dx; double dt;
 *   8 zero bytes
 * followed by phi_0..phi_3, mu_0, mu_1 as float32, each [z][y][x]
 * unpadded (24 bytes per cell).  FP64 values are rounded to nearest. */

/* Write the current state of `d` (after pf_init_fields) to the file `path`,
 * replacing it.  Synchronises.  The domain's second field copy serves as
 * staging space; the state and the step are unchanged.  INVALID_ARG for a
 * NULL argument, STATE before pf_init_fields, IO if the file cannot be
 * written. */
pf_status pf_checkpoint_save(pf_domain* d, const char* path);

/* Replace the state of `d` (after pf_set_params) with the checkpoint in
 * `path`, written for the same nx, ny, nz by a domain of either precision:
 * fields widened from float, step and window shifts from the header, so
 * t = step dt with this domain's dt.  Synchronises.  INVALID_ARG for a NULL
 * argument, a header that is not a checkpoint or a size mismatch, STATE
 * before pf_set_params or for a pack member, IO if the file cannot be
 * opened or its length is not header + 24 bytes per cell (the state is then
 * untouched) or a read fails part way; after a read or DEVICE error part
 * way the domain holds no state (step and read calls return STATE until
 * the next successful load or pf_init_fields). */
pf_status pf_checkpoint_load(pf_domain* d, const char* path);

/* Triangle mesh of the interface of phase `phase` (0..3): the surface
 * phi_phase = iso, iso finite, over the cubes of eight neighbouring cell
 * centres, periodic in x and y, open at the first and last z planes.
 * Vertices are in cell-index units (cell (x,y,z) at (x,y,z)); a cube past
 * the last column or row reaches the periodic image at x = nx or y = ny.
 * Each triangle is 9 floats (three vertices x, y, z), wound so that its
 * normal points out of the phase (towards phi_phase < iso).  `out` is a
 * caller-owned device buffer (base may be NULL when bytes is 0); up to
 * bytes / 36 triangles are written, in no fixed order.  *ntri receives the
 * total.  Returns INVALID_ARG (after filling *ntri and the buffer) when the
 * total exceeds the buffer, STATE before pf_init_fields.  Synchronises. */
pf_status pf_mesh_phase(pf_domain* d, int32_t phase, double iso, const pf_device_buffer* out,
                        int64_t* ntri);

/* Diagnostics of fields the caller holds in device memory, computed
 * without a domain and without allocating any memory.  For callers that
 * cannot allocate (code that must not call hipMalloc: serving loops with a
 * fixed footprint, harnesses that forbid allocation); not in the paper.
 * The sums are those pf_read_fields reports (conserved concentrations of
 * Eq. (3) under the frozen temperature, Sec. 2; sums of phi, the largest
 * |sum_a phi_a - 1|, phi range, non-finite cells), from the same kernel
 * arithmetic and reduction order, so for one state they are bitwise equal.
 *   desc:   sizes, precision (element type of `fields`) and dx.
 *   p:      only T0, G, v, zoff, TE, chi0, chi1, c0, c1 are read
 *           (T(z,t) = T0 + G (z dx + zoff - v t)).
 *   fields: device pointer to phi_0..3, mu_0, mu_1, each [z][y][x] with x
 *           fastest, no padding, one field after the other (6 nx ny nz
 *           elements); read only, still owned by the caller.
 *   t:      the time the fields belong to (finite).
 *   stream: hipStream_t to run on (NULL = null stream); the call waits for
 *           its own result before it returns.
 *   out:    filled like pf_read_fields' diag, with step = -1 and the item
 *           counts and window shifts 0.
 * Memory: partial sums go to a static device array of 480 x 10 + 10
 * doubles (38.5 KiB) that each GPU the library runs on keeps until the
 * process ends; its size does not depend on the domain, and every word a
 * call reads it has written first, so nothing needs clearing.  All calls
 * on one GPU share its array and it keeps the last call's values: calls
 * that overlapped on one GPU would race, so the library serialises them
 * with a host lock per device (the call returns only after its result is
 * back).  Errors: INVALID_ARG for null or misaligned
 * pointers, sizes <= 0, an unknown precision, fields beyond 2^62 bytes, a
 * non-finite t or dx <= 0; DEVICE for HIP errors; NONFINITE (outputs
 * filled) if any cell holds a NaN or Inf. */
pf_status pf_diag_fields_noalloc(const pf_domain_desc* desc, const pf_params* p,
                                 const void* fields, double t, void* stream,
                                 pf_diag* out);

/* Batched stepping (many independent domains of one precision).  Not in
 * the paper, which runs one large domain over many processes: batching
 * and serving of many independent solves are this library's use of one
 * GPU; each member still takes exactly the steps of Algorithm 1.  Each pack
 * step runs the per-plane coefficient kernel, the phi-sweep and the
 * mu-sweep once each for all member domains, over a flattened list of
 * (domain, tile) items; the step is captured once in a HIP graph and
 * replayed.  Members keep their own sizes, parameters, time and step count. */
pf_status pf_pack_create(int32_t prec, void* stream, int32_t max_domains,
                         pf_pack** out);
/* Add a domain (params and fields set, same precision) that should run
 * nsteps more steps; takes effect at the next pf_pack_step. */
pf_status pf_pack_add(pf_pack* pk, pf_domain* d, int64_t nsteps);
/* Run `rounds` pack steps; a member that has run its steps idles.  Reports
 * how many members have finished (they stay members until removed). */
pf_status pf_pack_step(pf_pack* pk, int64_t rounds, int32_t* n_finished);
/* Remaining steps of a member (0 = finished). */
pf_status pf_pack_remaining(pf_pack* pk, const pf_domain* d, int64_t* left);
pf_status pf_pack_remove(pf_pack* pk, pf_domain* d);
pf_status pf_pack_sync(pf_pack* pk);
void pf_pack_destroy(pf_pack* pk);

/* Kernel variant used by subsequent sweeps of every domain (Algorithm 1's
 * two kernels, in two implementations; not in the paper as a call):
 * 0 = one thread per cell evaluating all six faces ("direct"), 1 = z-marching
 * tiles that evaluate every face once and share it (default; Sec. 3.3,
 * staggered-value buffering).  Both compute the same model; the tests hold
 * both to the same tolerance.  INVALID_ARG for any other value. */
pf_status pf_set_variant(int32_t variant);

const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PFSOLVE_H */
