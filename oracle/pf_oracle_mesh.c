/*
 * pf_oracle_mesh.c -- plain CPU oracle of the interface meshes of the output
 * path (Sec. 3.2, Input/Output: one triangle mesh per phase, from a marching
 * cubes pass over phi, after Lorensen and Cline).
 *
 * TEST INFRASTRUCTURE ONLY (see pf_oracle.h).  It shares no code with the
 * HIP library.
 *
 * Reading taken (the paper gives no details beyond the method): the mesh of
 * phase a is the surface phi_a = iso over the cubes whose eight corners are
 * neighbouring cell centres, periodic in x and y, not extended past the
 * first and last z planes.  A corner is inside when phi_a > iso.  On every
 * cube face the surface enters and leaves across the face edges whose two
 * corners differ; each run of consecutive inside corners, walking the face
 * boundary, is cut off by one segment from the crossing after the run to
 * the crossing before it (so on a face whose inside corners lie on a
 * diagonal, the two are kept apart: the rule depends on the face alone and
 * two cubes sharing a face agree).  The segments of the six faces close into
 * loops; each loop, started at its lowest-numbered edge, is split into a fan
 * of triangles, wound so that the normal points out of the phase (towards
 * phi_a < iso).  A vertex on the edge between corners A and B (the lower
 * numbered first) lies at A + t (B - A), t = (iso - phi_A) / (phi_B - phi_A),
 * in FP64, then rounded to float.  Coordinates are cell indices (cell
 * (x, y, z) at (x, y, z)); a cube past the last x or y column reaches the
 * periodic image at nx or ny.
 *
 * The per-cube construction below walks the faces directly; it uses no
 * precomputed case table.
 */
#include <string.h>

#include "pf_oracle.h"

/* corner c of a cube sits at (c & 1, (c >> 1) & 1, (c >> 2) & 1) */
static int corner_bit(int c, int axis) { return (c >> axis) & 1; }

/* The edge between two corners that differ in one coordinate, numbered by
 * axis: x edges 0-3, y edges 4-7, z edges 8-11, each group ordered by the
 * remaining two coordinates (lower one fastest). */
static int edge_of(int a, int b) {
  const int d = a ^ b;
  const int axis = d == 1 ? 0 : (d == 2 ? 1 : 2);
  const int lo = a < b ? a : b;
  int r = 0, k = 0;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax == axis) continue;
    r |= corner_bit(lo, ax) << k;
    ++k;
  }
  return 4 * axis + r;
}

/* The two corners of edge e, lower first. */
static void edge_corners(int e, int* a, int* b) {
  const int axis = e / 4, r = e % 4;
  int lo = 0, k = 0;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax == axis) continue;
    lo |= ((r >> k) & 1) << ax;
    ++k;
  }
  *a = lo;
  *b = lo | (1 << axis);
}

/* Corners of each face in counter-clockwise order seen from outside the
 * cube: -x, +x, -y, +y, -z, +z. */
static const int kFace[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};

/* Triangles of one cube from the inside flags of its corners: loops of
 * edge numbers, fan-split.  Returns the number of triangles; tri[3 n] holds
 * their edges. */
static int cube_triangles(const int inside[8], int tri[3 * 12]) {
  int next[12];
  for (int e = 0; e < 12; ++e) next[e] = -1;
  for (int f = 0; f < 6; ++f) {
    const int* c = kFace[f];
    for (int i = 0; i < 4; ++i) {
      const int prev = (i + 3) % 4;
      if (!inside[c[i]] || inside[c[prev]]) continue;  /* a run starts at corner i */
      const int entry = edge_of(c[prev], c[i]);
      int j = i;
      while (inside[c[(j + 1) % 4]]) j = (j + 1) % 4;
      const int exit_ = edge_of(c[j], c[(j + 1) % 4]);
      next[exit_] = entry;
    }
  }
  int n = 0, used[12] = {0};
  for (int s = 0; s < 12; ++s) {
    if (next[s] < 0 || used[s]) continue;
    int loop[12], m = 0, e = s;
    do {
      used[e] = 1;
      loop[m++] = e;
      e = next[e];
    } while (e != s);
    for (int i = 1; i + 1 < m; ++i) {  /* normal out of the phase */
      tri[3 * n + 0] = loop[0];
      tri[3 * n + 1] = loop[i + 1];
      tri[3 * n + 2] = loop[i];
      ++n;
    }
  }
  return n;
}

int64_t orc_mesh_phase(const orc_grid* g, const double* phi, int32_t phase, double iso,
                       float* out, int64_t capacity) {
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
  const double* f = phi + (int64_t)phase * nx * ny * nz;
  int64_t count = 0;
  for (int64_t z = 0; z + 1 < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        double v[8];
        int inside[8], any_in = 0, any_out = 0;
        for (int c = 0; c < 8; ++c) {
          const int64_t cx = (x + corner_bit(c, 0)) % nx, cy = (y + corner_bit(c, 1)) % ny;
          const int64_t cz = z + corner_bit(c, 2);
          v[c] = f[(cz * ny + cy) * nx + cx];
          inside[c] = v[c] > iso;
          any_in |= inside[c];
          any_out |= !inside[c];
        }
        if (!any_in || !any_out) continue;
        int tri[3 * 12];
        const int n = cube_triangles(inside, tri);
        for (int k = 0; k < n; ++k, ++count) {
          if (count >= capacity) continue;
          for (int q = 0; q < 3; ++q) {
            int a, b;
            edge_corners(tri[3 * k + q], &a, &b);
            const double t = (iso - v[a]) / (v[b] - v[a]);
            const double p[3] = {(double)(x + corner_bit(a, 0)), (double)(y + corner_bit(a, 1)),
                                 (double)(z + corner_bit(a, 2))};
            const int axis = tri[3 * k + q] / 4;
            for (int d = 0; d < 3; ++d)
              out[9 * count + 3 * q + d] = (float)(d == axis ? p[d] + t : p[d]);
          }
        }
      }
  return count;
}
