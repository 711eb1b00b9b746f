/*
 * oracle.c -- plain, slow FP64 CPU oracle for the objectives and constraints of
 * multi-objective dual simplex-mesh deformable image registration
 * (Andreadis, Bosman, Alderliesten: "Multi-Objective Dual Simplex-Mesh Based
 * Deformable Image Registration for 3D Medical Images -- Proof of Concept").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the GPU library.
 *
 * Everything here is the plain definition written out: every tetrahedron, every
 * voxel of its bounding box, an exact point-in-tetrahedron test per voxel, FP64
 * barycentric mapping, FP64 trilinear sampling, FP64 sums.  No blocking, no spans,
 * no incremental evaluation.
 *
 * Conventions (readings of passages where the paper is silent):
 *   - grid 0 = source ("moving") grid on the source image, grid 1 = target
 *     ("fixed") grid on the target image (Sec. 2.1: a source image is registered
 *     onto a target image; forward = transformed source compared to target,
 *     Sec. 2.3.1).
 *   - voxel (i,j,k) has its centre at (i,j,k) in voxel units; each grid spans
 *     the box [-0.5, D-0.5] per axis.
 *   - coordinates live on a lattice of 1/128 voxel: u = (x + 0.5) * 128 is an
 *     integer in [0, 128*D], D <= 512, so |u| <= 2^16 and every orientation
 *     determinant below is an integer below 2^51: FP64 evaluates it exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LAT 128.0

/* flag bits of a candidate solution (constraint violations, Sec. 2.3.4) */
#define F_INV_MOVING 1u
#define F_INV_FIXED 2u
#define F_BORDER 4u
#define F_DOMAIN 8u
#define F_LATTICE 16u
#define F_NONFINITE 32u

typedef struct {
  int D[3];
  double sp[3];
  long V;
  double *img[2]; /* img[0] = source (moving), img[1] = target (fixed); [z][y][x] */
  int n[3];
  int P, C, T, E, max_star;
  int *tet;      /* [T][4] */
  int *edge;     /* [E][2] */
  int *ke;       /* [E] number of tetrahedra sharing the edge */
  int *tet_edge; /* [T][6] edge id of vertex pairs 01 02 03 12 13 23 */
  int *star_off; /* [P+1] */
  int *star;     /* [4T] tetrahedra incident to each point, ascending */
  double tau;
  int ng[2];     /* guidance points on the source image (0) and target image (1) */
  double *g[2];  /* [ng][3] lattice units */
  int *gc[2];    /* correspondence id per point */
  int hard_threshold;   /* study flag: threshold the sampled value instead of interpolating the mask */
  int abs_deformation;  /* study flag: |dL| instead of dL^2 */
} ref_problem;

/* ---------------------------------------------------------------- topology */

/* Sec. 2.1 and Fig. 1(A,B): each cube of 8 grid points is split into 6
 * tetrahedra; cubes are mirrored inside every 2x2x2 group.  Reading: the 6
 * tetrahedra are the monotone lattice paths from local corner (0,0,0) to
 * (1,1,1), one per axis permutation (lexicographic order xyz xzy yxz yzx zxy
 * zyx), and the local corner l of cube (ci,cj,ck) is the global point
 * (ci + (lx ^ (ci&1)), cj + (ly ^ (cj&1)), ck + (lz ^ (ck&1))). */
static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static int pidx(const int n[3], int i, int j, int k) { return i + n[0] * (j + n[1] * k); }

/* orientation determinant det[b-a; c-a; d-a] (positive = right-handed) */
static double orient3d(const double a[3], const double b[3], const double c[3], const double d[3]) {
  double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
  double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
  double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
  return bx * (cy * dz - cz * dy) - by * (cx * dz - cz * dx) + bz * (cx * dy - cy * dx);
}

double ref_orient3d(const double *a, const double *b, const double *c, const double *d) {
  return orient3d(a, b, c, d);
}

static int cmp_pair(const void *x, const void *y) {
  const int *a = (const int *)x, *b = (const int *)y;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

static void build_topology(ref_problem *p) {
  const int *n = p->n;
  p->P = n[0] * n[1] * n[2];
  p->C = (n[0] - 1) * (n[1] - 1) * (n[2] - 1);
  p->T = 6 * p->C;
  p->tet = (int *)malloc(sizeof(int) * 4 * p->T);
  for (int ck = 0; ck < n[2] - 1; ++ck)
    for (int cj = 0; cj < n[1] - 1; ++cj)
      for (int ci = 0; ci < n[0] - 1; ++ci) {
        int cube = ci + (n[0] - 1) * (cj + (n[1] - 1) * ck);
        int m[3] = {ci & 1, cj & 1, ck & 1};
        int base[3] = {ci, cj, ck};
        for (int s = 0; s < 6; ++s) {
          int l[3] = {0, 0, 0};
          int v[4];
          double pos[4][3];
          for (int step = 0; step < 4; ++step) {
            if (step > 0) l[PERM[s][step - 1]] = 1;
            int g[3];
            for (int a = 0; a < 3; ++a) g[a] = base[a] + (l[a] ^ m[a]);
            v[step] = pidx(n, g[0], g[1], g[2]);
            for (int a = 0; a < 3; ++a) pos[step][a] = g[a];
          }
          /* keep every tetrahedron positively oriented on the undeformed grid */
          if (orient3d(pos[0], pos[1], pos[2], pos[3]) < 0) {
            int t = v[2];
            v[2] = v[3];
            v[3] = t;
          }
          for (int q = 0; q < 4; ++q) p->tet[4 * (6 * cube + s) + q] = v[q];
        }
      }
  /* unique edges (Sec. 2.3.2) and the number of tetrahedra sharing each */
  static const int VP[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  int *pairs = (int *)malloc(sizeof(int) * 2 * 6 * p->T);
  for (int t = 0; t < p->T; ++t)
    for (int e = 0; e < 6; ++e) {
      int a = p->tet[4 * t + VP[e][0]], b = p->tet[4 * t + VP[e][1]];
      pairs[2 * (6 * t + e)] = a < b ? a : b;
      pairs[2 * (6 * t + e) + 1] = a < b ? b : a;
    }
  int *sorted = (int *)malloc(sizeof(int) * 2 * 6 * p->T);
  memcpy(sorted, pairs, sizeof(int) * 2 * 6 * p->T);
  qsort(sorted, 6 * p->T, 2 * sizeof(int), cmp_pair);
  p->edge = (int *)malloc(sizeof(int) * 2 * 6 * p->T);
  p->ke = (int *)malloc(sizeof(int) * 6 * p->T);
  p->E = 0;
  for (int i = 0; i < 6 * p->T; ++i) {
    if (p->E > 0 && sorted[2 * i] == p->edge[2 * (p->E - 1)] && sorted[2 * i + 1] == p->edge[2 * (p->E - 1) + 1]) {
      p->ke[p->E - 1]++;
      continue;
    }
    p->edge[2 * p->E] = sorted[2 * i];
    p->edge[2 * p->E + 1] = sorted[2 * i + 1];
    p->ke[p->E] = 1;
    p->E++;
  }
  p->tet_edge = (int *)malloc(sizeof(int) * 6 * p->T);
  for (int i = 0; i < 6 * p->T; ++i) {
    /* binary search for the pair */
    int lo = 0, hi = p->E - 1;
    while (lo < hi) {
      int mid = (lo + hi) / 2;
      if (cmp_pair(&p->edge[2 * mid], &pairs[2 * i]) < 0)
        lo = mid + 1;
      else
        hi = mid;
    }
    p->tet_edge[i] = lo;
  }
  free(sorted);
  free(pairs);
  /* star of each point: the tetrahedra that must be re-evaluated when it moves (Sec. 2.2) */
  p->star_off = (int *)calloc(p->P + 1, sizeof(int));
  for (int t = 0; t < p->T; ++t)
    for (int q = 0; q < 4; ++q) p->star_off[p->tet[4 * t + q] + 1]++;
  for (int i = 0; i < p->P; ++i) p->star_off[i + 1] += p->star_off[i];
  p->star = (int *)malloc(sizeof(int) * 4 * p->T);
  int *fill = (int *)calloc(p->P, sizeof(int));
  for (int t = 0; t < p->T; ++t)
    for (int q = 0; q < 4; ++q) {
      int v = p->tet[4 * t + q];
      p->star[p->star_off[v] + fill[v]++] = t;
    }
  free(fill);
  p->max_star = 0;
  for (int i = 0; i < p->P; ++i) {
    int s = p->star_off[i + 1] - p->star_off[i];
    if (s > p->max_star) p->max_star = s;
  }
}

/* ---------------------------------------------------------------- lattice */

/* voxel-unit coordinate -> lattice integer (as a double); returns flag bits */
static unsigned to_lattice(double x, int D, double *u) {
  if (!isfinite(x)) return F_NONFINITE;
  double v = (x + 0.5) * LAT;
  *u = v;
  if (v != floor(v)) return F_LATTICE;
  if (v < 0 || v > LAT * D) return F_DOMAIN;
  return 0;
}

/* ---------------------------------------------------------------- create */

ref_problem *ref_create(const int *D, const double *sp, const float *moving, const float *fixed, const int *n,
                        double tau, int n_mov, const float *g_mov, const int *c_mov, int n_fix, const float *g_fix,
                        const int *c_fix, int hard_threshold, int abs_deformation) {
  ref_problem *p = (ref_problem *)calloc(1, sizeof(ref_problem));
  for (int a = 0; a < 3; ++a) {
    p->D[a] = D[a];
    p->sp[a] = sp[a];
    p->n[a] = n[a];
  }
  p->V = (long)D[0] * D[1] * D[2];
  for (int g = 0; g < 2; ++g) {
    const float *src = g == 0 ? moving : fixed;
    p->img[g] = (double *)malloc(sizeof(double) * p->V);
    for (long i = 0; i < p->V; ++i) p->img[g][i] = src[i];
  }
  p->tau = tau;
  p->hard_threshold = hard_threshold;
  p->abs_deformation = abs_deformation;
  build_topology(p);
  int ng[2] = {n_mov, n_fix};
  const float *gs[2] = {g_mov, g_fix};
  const int *cs[2] = {c_mov, c_fix};
  for (int g = 0; g < 2; ++g) {
    p->ng[g] = ng[g];
    p->g[g] = (double *)malloc(sizeof(double) * 3 * (ng[g] > 0 ? ng[g] : 1));
    p->gc[g] = (int *)malloc(sizeof(int) * (ng[g] > 0 ? ng[g] : 1));
    for (int i = 0; i < ng[g]; ++i) {
      for (int a = 0; a < 3; ++a) p->g[g][3 * i + a] = rint(((double)gs[g][3 * i + a] + 0.5) * LAT);
      p->gc[g][i] = cs[g][i];
    }
  }
  return p;
}

void ref_destroy(ref_problem *p) {
  if (!p) return;
  for (int g = 0; g < 2; ++g) {
    free(p->img[g]);
    free(p->g[g]);
    free(p->gc[g]);
  }
  free(p->tet);
  free(p->edge);
  free(p->ke);
  free(p->tet_edge);
  free(p->star_off);
  free(p->star);
  free(p);
}

void ref_counts(const ref_problem *p, int *out) {
  out[0] = p->P;
  out[1] = p->T;
  out[2] = p->E;
  out[3] = p->max_star;
}
void ref_tets(const ref_problem *p, int *out) { memcpy(out, p->tet, sizeof(int) * 4 * p->T); }
void ref_edges(const ref_problem *p, int *out, int *ke) {
  memcpy(out, p->edge, sizeof(int) * 2 * p->E);
  memcpy(ke, p->ke, sizeof(int) * p->E);
}
void ref_star(const ref_problem *p, int *off, int *st) {
  memcpy(off, p->star_off, sizeof(int) * (p->P + 1));
  memcpy(st, p->star, sizeof(int) * 4 * p->T);
}

/* undeformed grid: point i of n on an axis of D voxels sits at lattice
 * round_half_up(i * 128 * D / (n - 1)) (reading: the grid spans the image box). */
void ref_identity(const ref_problem *p, float *X) {
  for (int k = 0; k < p->n[2]; ++k)
    for (int j = 0; j < p->n[1]; ++j)
      for (int i = 0; i < p->n[0]; ++i) {
        int idx[3] = {i, j, k};
        int v = pidx(p->n, i, j, k);
        for (int a = 0; a < 3; ++a) {
          long num = 2L * idx[a] * 128L * p->D[a] + (p->n[a] - 1);
          long u = num / (2L * (p->n[a] - 1));
          X[3 * v + a] = (float)((double)u / LAT - 0.5);
        }
      }
}

/* ---------------------------------------------------------------- predicate */

/* Sec. 2.3.1 (rasterisation with the top-left rule, footnote), generalised to
 * 3-D: point U (lattice) lies in the positively oriented tetrahedron V iff for
 * every face i the orientation o_i (U replacing vertex i) is > 0, or it is 0 and
 * the first non-zero of its change along +x, +y, +z is > 0.  Writes o_i. */
static int inside(const double V[4][3], const double U[3], double o[4]) {
  double vol = orient3d(V[0], V[1], V[2], V[3]);
  if (vol <= 0) return 0;
  for (int i = 0; i < 4; ++i) {
    double W[4][3];
    memcpy(W, V, sizeof(W));
    for (int a = 0; a < 3; ++a) W[i][a] = U[a];
    o[i] = orient3d(W[0], W[1], W[2], W[3]);
    if (o[i] > 0) continue;
    if (o[i] < 0) return 0;
    int decided = 0;
    for (int a = 0; a < 3 && !decided; ++a) {
      W[i][a] = U[a] + 1.0;
      double g = orient3d(W[0], W[1], W[2], W[3]);
      W[i][a] = U[a];
      if (g > 0) decided = 1;
      else if (g < 0) return 0;
    }
    if (!decided) return 0;
  }
  return 1;
}

int ref_inside(const double *V, const double *U) {
  double Vv[4][3], o[4];
  memcpy(Vv, V, sizeof(Vv));
  return inside(Vv, U, o);
}

/* gather the 4 vertices of tetrahedron t of grid g from coordinates Xg [P][3]
 * (voxel units) into lattice and voxel units; returns flag bits */
static unsigned tet_vertices(const ref_problem *p, const float *Xg, int t, double L[4][3], double Vx[4][3]) {
  unsigned f = 0;
  for (int q = 0; q < 4; ++q) {
    int v = p->tet[4 * t + q];
    for (int a = 0; a < 3; ++a) {
      double x = Xg[3 * v + a];
      Vx[q][a] = x;
      f |= to_lattice(x, p->D[a], &L[q][a]);
    }
  }
  return f;
}

/* inclusive voxel index range covered by the lattice interval [lo, hi] */
static void vox_range(double lo, double hi, int D, int *a, int *b) {
  /* voxel i has lattice centre 128 i + 64 */
  *a = (int)ceil((lo - 64.0) / LAT);
  *b = (int)floor((hi - 64.0) / LAT);
  if (*a < 0) *a = 0;
  if (*b > D - 1) *b = D - 1;
}

/* brute-force owner map of one grid: owner[v] = the tetrahedron containing voxel
 * centre v (-1 if none), count[v] = how many contain it.  Sec. 2.3.1. */
void ref_owner_bruteforce(const ref_problem *p, const float *Xg, int *owner, int *count) {
  double (*L)[4][3] = malloc(sizeof(double) * 12 * p->T);
  double Vx[4][3];
  int *ok = malloc(sizeof(int) * p->T);
  for (int t = 0; t < p->T; ++t) ok[t] = tet_vertices(p, Xg, t, L[t], Vx) == 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < p->D[2]; ++k)
    for (int j = 0; j < p->D[1]; ++j)
      for (int i = 0; i < p->D[0]; ++i) {
        long v = i + (long)p->D[0] * (j + (long)p->D[1] * k);
        double U[3] = {LAT * i + 64, LAT * j + 64, LAT * k + 64}, o[4];
        owner[v] = -1;
        count[v] = 0;
        for (int t = 0; t < p->T; ++t)
          if (ok[t] && inside(L[t], U, o)) {
            if (owner[v] < 0) owner[v] = t;
            count[v]++;
          }
      }
  free(ok);
  free(L);
}

/* voxels of tetrahedron t (grid coordinates Xg) by scanning its bounding box */
int ref_tet_voxels(const ref_problem *p, const float *Xg, int t, long *out, int cap) {
  double L[4][3], Vx[4][3], o[4];
  if (tet_vertices(p, Xg, t, L, Vx)) return 0;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    double mn = L[0][a], mx = L[0][a];
    for (int q = 1; q < 4; ++q) {
      if (L[q][a] < mn) mn = L[q][a];
      if (L[q][a] > mx) mx = L[q][a];
    }
    vox_range(mn, mx, p->D[a], &lo[a], &hi[a]);
  }
  int cnt = 0;
  for (int k = lo[2]; k <= hi[2]; ++k)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int i = lo[0]; i <= hi[0]; ++i) {
        double U[3] = {LAT * i + 64, LAT * j + 64, LAT * k + 64};
        if (inside(L, U, o)) {
          if (cnt < cap) out[cnt] = i + (long)p->D[0] * (j + (long)p->D[1] * k);
          cnt++;
        }
      }
  return cnt;
}

/* ---------------------------------------------------------------- sampling */

static double empty_of(const ref_problem *p, double v) { return v <= p->tau ? 1.0 : 0.0; }

/* trilinear interpolation of image g (mask=0) or of its empty-indicator (mask=1)
 * at voxel-unit position x, clamped to [0, D-1] per axis. */
static double trilinear(const ref_problem *p, int g, const double x[3], int mask) {
  int i0[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double c = x[a];
    if (c < 0) c = 0;
    if (c > p->D[a] - 1) c = p->D[a] - 1;
    int i = (int)floor(c);
    if (i > p->D[a] - 2) i = p->D[a] - 2;
    i0[a] = i;
    f[a] = c - i;
  }
  double acc = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        double w = (dx ? f[0] : 1 - f[0]) * (dy ? f[1] : 1 - f[1]) * (dz ? f[2] : 1 - f[2]);
        long v = (i0[0] + dx) + (long)p->D[0] * ((i0[1] + dy) + (long)p->D[1] * (i0[2] + dz));
        double val = p->img[g][v];
        acc += w * (mask ? empty_of(p, val) : val);
      }
  return acc;
}

double ref_trilinear(const ref_problem *p, int g, const double *x, int mask) { return trilinear(p, g, x, mask); }

/* Sec. 2.3.1: contribution of one pair of corresponding voxels.  Squared
 * intensity difference; a mismatch between empty (black) and non-empty (grey)
 * counts as the maximal difference 1.  Reading: the empty indicator of the
 * sampled position is interpolated like the intensity, m = |e_a - e_b| blends
 * between the two cases. */
static double contribution(const ref_problem *p, double a, double b, double eb) {
  double ea = empty_of(p, a);
  if (p->hard_threshold) {
    double m = (ea != empty_of(p, b)) ? 1.0 : 0.0;
    return m ? 1.0 : (a - b) * (a - b);
  }
  double m = fabs(ea - eb);
  return (1 - m) * (a - b) * (a - b) + m;
}

/* dissimilarity sum over the voxels of one tetrahedron in one direction:
 * voxels of image `own` inside the tetrahedron of grid `own` are mapped with
 * barycentric coordinates to the same tetrahedron of the other grid and compared
 * with the other image there. */
static double sim_direction(const ref_problem *p, int own, const double Lown[4][3], const double Xoth[4][3],
                            long *nvox) {
  double vol = orient3d(Lown[0], Lown[1], Lown[2], Lown[3]);
  if (vol <= 0) return 0;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    double mn = Lown[0][a], mx = Lown[0][a];
    for (int q = 1; q < 4; ++q) {
      if (Lown[q][a] < mn) mn = Lown[q][a];
      if (Lown[q][a] > mx) mx = Lown[q][a];
    }
    vox_range(mn, mx, p->D[a], &lo[a], &hi[a]);
  }
  double sum = 0;
  for (int k = lo[2]; k <= hi[2]; ++k)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int i = lo[0]; i <= hi[0]; ++i) {
        double U[3] = {LAT * i + 64, LAT * j + 64, LAT * k + 64}, o[4];
        if (!inside(Lown, U, o)) continue;
        double x[3] = {0, 0, 0};
        for (int q = 0; q < 4; ++q) {
          double lam = o[q] / vol;
          for (int a = 0; a < 3; ++a) x[a] += lam * Xoth[q][a];
        }
        long v = i + (long)p->D[0] * (j + (long)p->D[1] * k);
        double a = p->img[own][v];
        double b = trilinear(p, 1 - own, x, 0);
        double eb = trilinear(p, 1 - own, x, 1);
        sum += contribution(p, a, b, eb);
        (*nvox)++;
      }
  return sum;
}

static double len_mm(const ref_problem *p, const double a[3], const double b[3]) {
  double s = 0;
  for (int c = 0; c < 3; ++c) {
    double d = (a[c] - b[c]) * p->sp[c];
    s += d * d;
  }
  return sqrt(s);
}

/* Sec. 2.3.2: Hooke's-law energy of one tetrahedron: edge-length differences
 * between source and target grid (each edge weighted 1/k_e so that summing over
 * all tetrahedra counts each edge once) plus the 4 spoke edges from each vertex
 * to the centroid of its opposite face.  Reading: squared differences in mm. */
static double deformation_tet(const ref_problem *p, int t, const double S[4][3], const double Tg[4][3]) {
  static const int VP[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  double sum = 0;
  for (int e = 0; e < 6; ++e) {
    double d = len_mm(p, S[VP[e][0]], S[VP[e][1]]) - len_mm(p, Tg[VP[e][0]], Tg[VP[e][1]]);
    double w = 1.0 / p->ke[p->tet_edge[6 * t + e]];
    sum += w * (p->abs_deformation ? fabs(d) : d * d);
  }
  for (int q = 0; q < 4; ++q) {
    double cS[3] = {0, 0, 0}, cT[3] = {0, 0, 0};
    for (int r = 0; r < 4; ++r)
      if (r != q)
        for (int a = 0; a < 3; ++a) {
          cS[a] += S[r][a] / 3.0;
          cT[a] += Tg[r][a] / 3.0;
        }
    double d = len_mm(p, S[q], cS) - len_mm(p, Tg[q], cT);
    sum += p->abs_deformation ? fabs(d) : d * d;
  }
  return sum;
}

/* Sec. 2.3.3: guidance points of image g that lie in tetrahedron t of grid g
 * are transformed into the other image; each contributes the squared mm
 * distance to the nearest point of the same correspondence there. */
static double guidance_tet(const ref_problem *p, const double L[2][4][3], const double X[2][4][3]) {
  double sum = 0;
  for (int g = 0; g < 2; ++g) {
    for (int i = 0; i < p->ng[g]; ++i) {
      double o[4];
      if (!inside(L[g], &p->g[g][3 * i], o)) continue;
      double vol = orient3d(L[g][0], L[g][1], L[g][2], L[g][3]);
      double x[3] = {0, 0, 0};
      for (int q = 0; q < 4; ++q)
        for (int a = 0; a < 3; ++a) x[a] += o[q] / vol * X[1 - g][q][a];
      double best = INFINITY;
      for (int j = 0; j < p->ng[1 - g]; ++j) {
        if (p->gc[1 - g][j] != p->gc[g][i]) continue;
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = p->g[1 - g][3 * j + a] / LAT - 0.5;
        double d = len_mm(p, x, r);
        if (d < best) best = d;
      }
      if (isfinite(best)) sum += best * best;
    }
  }
  return sum;
}

/* raw (un-normalised) terms {dissimilarity, deformation, guidance} of one
 * tetrahedron given both grids' coordinates ([2][P][3]) */
static void tet_terms(const ref_problem *p, const float *X2, int t, double out[3], long *nvox) {
  double L[2][4][3], Xv[2][4][3];
  unsigned f = 0;
  for (int g = 0; g < 2; ++g) f |= tet_vertices(p, X2 + (long)g * 3 * p->P, t, L[g], Xv[g]);
  out[0] = out[1] = out[2] = 0;
  if (f) return;
  /* forward: target voxels in the target grid -> source image; backward: the reverse */
  out[0] = sim_direction(p, 1, L[1], Xv[0], nvox) + sim_direction(p, 0, L[0], Xv[1], nvox);
  out[1] = deformation_tet(p, t, Xv[0], Xv[1]);
  out[2] = guidance_tet(p, L, Xv);
}

/* constraint flags (Sec. 2.3.4) of the given points and tetrahedra */
static unsigned check(const ref_problem *p, const float *X2, const int *pts, int npts, const int *tets, int ntets,
                      int *first_bad) {
  unsigned f = 0;
  for (int q = 0; q < npts; ++q) {
    int v = pts[q];
    int idx[3] = {v % p->n[0], (v / p->n[0]) % p->n[1], v / (p->n[0] * p->n[1])};
    for (int g = 0; g < 2; ++g)
      for (int a = 0; a < 3; ++a) {
        double u;
        unsigned fa = to_lattice(X2[(long)g * 3 * p->P + 3 * v + a], p->D[a], &u);
        f |= fa;
        if (fa) continue;
        /* border points move only within their border (pinned axes) */
        if (idx[a] == 0 && u != 0) f |= F_BORDER;
        if (idx[a] == p->n[a] - 1 && u != LAT * p->D[a]) f |= F_BORDER;
      }
  }
  for (int q = 0; q < ntets; ++q) {
    int t = tets[q];
    for (int g = 0; g < 2; ++g) {
      double L[4][3], Vx[4][3];
      if (tet_vertices(p, X2 + (long)g * 3 * p->P, t, L, Vx)) continue;
      if (orient3d(L[0], L[1], L[2], L[3]) <= 0) {
        f |= g == 0 ? F_INV_MOVING : F_INV_FIXED;
        if (first_bad && (*first_bad < 0 || t < *first_bad)) *first_bad = t;
      }
    }
  }
  return f;
}

static double norm_sim(const ref_problem *p) { return 1.0 / (2.0 * (double)p->V); }
static double norm_def(const ref_problem *p) { return 1.0 / (double)(p->E + 4 * p->T); }
static double norm_guid(const ref_problem *p) {
  int n = p->ng[0] + p->ng[1];
  return n > 0 ? 1.0 / n : 0.0;
}

/* ---------------------------------------------------------------- entry points */

/* Sec. 2.3.4: fold / constraint check of whole solutions X [S][2][P][3] */
void ref_fold_check(const ref_problem *p, int S, const float *X, uint32_t *flags, int *first_bad) {
  int *pts = malloc(sizeof(int) * p->P), *tets = malloc(sizeof(int) * p->T);
  for (int i = 0; i < p->P; ++i) pts[i] = i;
  for (int i = 0; i < p->T; ++i) tets[i] = i;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < S; ++s) {
    int fb = -1;
    flags[s] = check(p, X + (long)s * 6 * p->P, pts, p->P, tets, p->T, &fb);
    if (first_bad) first_bad[s] = fb;
  }
  free(pts);
  free(tets);
}

/* Sec. 2.3: full evaluation of every solution: objectives [S][3] normalised,
 * flags [S], optional raw per-tetrahedron terms [S][T][3] */
void ref_eval_full(const ref_problem *p, int S, const float *X, double *obj, uint32_t *flags, double *tet_terms_out,
                   long *nvox_out) {
  ref_fold_check(p, S, X, flags, NULL);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < S; ++s) {
    double acc[3] = {0, 0, 0};
    long nv = 0;
    for (int t = 0; t < p->T; ++t) {
      double tt[3];
      tet_terms(p, X + (long)s * 6 * p->P, t, tt, &nv);
      for (int c = 0; c < 3; ++c) acc[c] += tt[c];
      if (tet_terms_out)
        for (int c = 0; c < 3; ++c) tet_terms_out[((long)s * p->T + t) * 3 + c] = tt[c];
    }
    obj[3 * s + 0] = acc[0] * norm_sim(p);
    obj[3 * s + 1] = acc[1] * norm_def(p);
    obj[3 * s + 2] = acc[2] * norm_guid(p);
    if (nvox_out) nvox_out[s] = nv;
  }
}

static int cmp_int(const void *a, const void *b) { return *(const int *)a - *(const int *)b; }

/* the tetrahedra affected by moving the points of one FOS element: the union of
 * their stars, ascending (Sec. 2.2: tetrahedra to re-evaluate when a point moves) */
static int affected(const ref_problem *p, const int *pts, int npts, int *out) {
  int n = 0;
  for (int q = 0; q < npts; ++q)
    for (int i = p->star_off[pts[q]]; i < p->star_off[pts[q] + 1]; ++i) out[n++] = p->star[i];
  qsort(out, n, sizeof(int), cmp_int);
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (m == 0 || out[m - 1] != out[i]) out[m++] = out[i];
  return m;
}

/* Sec. 2.2-2.3: partial evaluation.  For every solution s and FOS element f the
 * candidate coordinates cand [S][fos_off[F]][2][3] replace the element's points
 * in both grids; part_new / part_old [S][F][3] are the normalised sums over the
 * affected tetrahedra of the candidate and current terms (part_old from
 * tet_terms_in [S][T][3] when given).  flags [S][F], nvox [S][F] = voxels
 * sampled for the candidate. */
void ref_eval_partial(const ref_problem *p, int S, const float *X, int F, const int *fos_off, const int *fos_pts,
                      const float *cand, const double *tet_terms_in, double *part_old, double *part_new,
                      uint32_t *flags, long *nvox) {
  int ncand = fos_off[F];
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int s = 0; s < S; ++s)
    for (int f = 0; f < F; ++f) {
      const float *Xs = X + (long)s * 6 * p->P;
      float *Xn = malloc(sizeof(float) * 6 * p->P);
      memcpy(Xn, Xs, sizeof(float) * 6 * p->P);
      int np = fos_off[f + 1] - fos_off[f];
      const int *pts = fos_pts + fos_off[f];
      for (int q = 0; q < np; ++q)
        for (int g = 0; g < 2; ++g)
          for (int a = 0; a < 3; ++a)
            Xn[(long)g * 3 * p->P + 3 * pts[q] + a] = cand[(((long)s * ncand + fos_off[f] + q) * 2 + g) * 3 + a];
      int *A = malloc(sizeof(int) * (np * p->max_star + 1));
      int na = affected(p, pts, np, A);
      /* constraint check over the affected tetrahedra and their vertices */
      int *vs = malloc(sizeof(int) * 4 * (na + 1));
      for (int i = 0; i < na; ++i)
        for (int q = 0; q < 4; ++q) vs[4 * i + q] = p->tet[4 * A[i] + q];
      long fi = (long)s * F + f;
      flags[fi] = check(p, Xn, vs, 4 * na, A, na, NULL);
      double accn[3] = {0, 0, 0}, acco[3] = {0, 0, 0};
      long nv = 0, nvo = 0;
      for (int i = 0; i < na; ++i) {
        double tt[3];
        tet_terms(p, Xn, A[i], tt, &nv);
        for (int c = 0; c < 3; ++c) accn[c] += tt[c];
        if (tet_terms_in) {
          for (int c = 0; c < 3; ++c) acco[c] += tet_terms_in[((long)s * p->T + A[i]) * 3 + c];
        } else {
          tet_terms(p, Xs, A[i], tt, &nvo);
          for (int c = 0; c < 3; ++c) acco[c] += tt[c];
        }
      }
      double nrm[3] = {norm_sim(p), norm_def(p), norm_guid(p)};
      for (int c = 0; c < 3; ++c) {
        part_new[fi * 3 + c] = accn[c] * nrm[c];
        part_old[fi * 3 + c] = acco[c] * nrm[c];
      }
      if (nvox) nvox[fi] = nv;
      free(vs);
      free(A);
      free(Xn);
    }
}

/* raw terms of a single tetrahedron for a single solution [2][P][3] (test hook) */
void ref_tet_terms(const ref_problem *p, const float *X2, int t, double *out) {
  long nv = 0;
  tet_terms(p, X2, t, out, &nv);
}

void ref_normalisers(const ref_problem *p, double *out) {
  out[0] = norm_sim(p);
  out[1] = norm_def(p);
  out[2] = norm_guid(p);
}

/* ------------------------------------------------------------------ transformation
 * Sec. 2.1: the two grids define a piecewise-affine map between the images;
 * each tetrahedron of one grid maps affinely onto the same tetrahedron of the
 * other.  Sec. 3 (Fig. 2) shows its result as a transformed source image and a
 * deformation vector field (DVF).  For every voxel v of image `own`, found in
 * its tetrahedron of grid `own` with the exact test used for the objectives,
 * x(v) = sum_q lambda_q(v) X_other[q] is the position it maps to in the other
 * image (voxel units).  Outputs (either may be NULL):
 *   dvf [V][3]  x(v) - v, in voxel units;
 *   warped [V]  the other image sampled at x(v) (trilinear, clamped), i.e. for
 *               own = 1 the transformed source image on the target grid.
 * Voxels inside no tetrahedron (only possible for an infeasible pair) stay NaN.
 * X2 is one solution [2][P][3]. */
void ref_transform(const ref_problem *p, int own, const float *X2, double *dvf, double *warped) {
  for (long v = 0; v < p->V; ++v) {
    if (dvf)
      for (int a = 0; a < 3; ++a) dvf[3 * v + a] = NAN;
    if (warped) warped[v] = NAN;
  }
  const float *Xo = X2 + (size_t)own * 3 * p->P, *Xt = X2 + (size_t)(1 - own) * 3 * p->P;
  for (int t = 0; t < p->T; ++t) {
    double Lown[4][3], Vown[4][3], Loth[4][3], Xoth[4][3];
    if (tet_vertices(p, Xo, t, Lown, Vown) || tet_vertices(p, Xt, t, Loth, Xoth)) continue;
    double vol = orient3d(Lown[0], Lown[1], Lown[2], Lown[3]);
    if (vol <= 0) continue;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      double mn = Lown[0][a], mx = Lown[0][a];
      for (int q = 1; q < 4; ++q) {
        if (Lown[q][a] < mn) mn = Lown[q][a];
        if (Lown[q][a] > mx) mx = Lown[q][a];
      }
      vox_range(mn, mx, p->D[a], &lo[a], &hi[a]);
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double U[3] = {LAT * i + 64, LAT * j + 64, LAT * k + 64}, o[4];
          if (!inside(Lown, U, o)) continue;
          double x[3] = {0, 0, 0};
          for (int q = 0; q < 4; ++q)
            for (int a = 0; a < 3; ++a) x[a] += o[q] / vol * Xoth[q][a];
          long v = i + (long)p->D[0] * (j + (long)p->D[1] * k);
          if (dvf) {
            dvf[3 * v + 0] = x[0] - i;
            dvf[3 * v + 1] = x[1] - j;
            dvf[3 * v + 2] = x[2] - k;
          }
          if (warped) warped[v] = trilinear(p, 1 - own, x, 0);
        }
  }
}

/* ------------------------------------------------------------------ refinement
 * Sec. 2.4 (grid multi-resolution): every cube of both grids is split into 8
 * cubes by adding a point in the middle of each cube edge, in the middle of
 * each face and at the cube's centre.  A grid of n points per axis becomes one
 * of 2n-1 points per axis: fine point (I,J,K) is the mean of the coarse points
 * (i,j,k) with i in {floor(I/2), ceil(I/2)} (and likewise for j, k), i.e. of 1
 * (a coarse point), 2 (edge middle), 4 (face middle) or 8 (cube centre) points.
 * Readings: the face middle and the centre are the means of the corners (the
 * faces of a deformed cube need not be planar); the mean is rounded to the
 * 1/128-voxel lattice, half to even.  Xc [S][2][Pc][3] -> Xf [S][2][Pf][3]. */
void ref_refine(const int *nc, int S, const float *Xc, float *Xf) {
  const int nf[3] = {2 * nc[0] - 1, 2 * nc[1] - 1, 2 * nc[2] - 1};
  const long Pc = (long)nc[0] * nc[1] * nc[2], Pf = (long)nf[0] * nf[1] * nf[2];
  for (int s = 0; s < S; ++s)
    for (int g = 0; g < 2; ++g)
      for (int K = 0; K < nf[2]; ++K)
        for (int J = 0; J < nf[1]; ++J)
          for (int I = 0; I < nf[0]; ++I) {
            const int is[2] = {I / 2, (I + 1) / 2}, js[2] = {J / 2, (J + 1) / 2}, ks[2] = {K / 2, (K + 1) / 2};
            double sum[3] = {0, 0, 0};
            int cnt = 0;
            /* the distinct coarse corners: index pairs collapse where I, J or K is even */
            for (int a = 0; a < (I % 2 ? 2 : 1); ++a)
              for (int b = 0; b < (J % 2 ? 2 : 1); ++b)
                for (int c = 0; c < (K % 2 ? 2 : 1); ++c) {
                  const float *x = Xc + (((long)s * 2 + g) * Pc + pidx(nc, is[a], js[b], ks[c])) * 3;
                  for (int d = 0; d < 3; ++d) sum[d] += ((double)x[d] + 0.5) * 128.0; /* lattice units */
                  ++cnt;
                }
            float *y = Xf + (((long)s * 2 + g) * Pf + pidx(nf, I, J, K)) * 3;
            for (int d = 0; d < 3; ++d) y[d] = (float)(nearbyint(sum[d] / cnt) / 128.0 - 0.5);
          }
}

/* ------------------------------------------------------- literal fold test
 * Sec. 2.3.4 as the paper states it (an oracle-only comparison with the exact
 * orientation test the library uses): an interior grid point must lie inside
 * the closed surface formed by the faces opposite it of its surrounding
 * tetrahedra, tested by casting a ray and counting triangle crossings; a point
 * on one border plane must lie inside the polygon formed, in that plane, by
 * the edges opposite it of the border faces of its surrounding tetrahedra,
 * tested by casting a ray in the plane and counting segment crossings.
 * Readings: points on a border edge must lie strictly between their two
 * neighbours on that edge; corners are fixed.  Arithmetic is exact: lattice
 * integers and 128-bit determinants; a ray that meets an edge or vertex
 * exactly is replaced by another direction.  Returns, per solution and grid,
 * the number of points that violate the test. */
typedef __int128 i128;

static i128 orient_i(const long a[3], const long b[3], const long c[3], const long d[3]) {
  const i128 bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
  const i128 cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
  const i128 dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
  return bx * (cy * dz - cz * dy) - by * (cx * dz - cz * dx) + bz * (cx * dy - cy * dx);
}

static int sgn(i128 v) { return v > 0 ? 1 : (v < 0 ? -1 : 0); }

/* does segment PQ cross triangle ABC?  returns 1 / 0, or -1 when degenerate */
static int seg_tri(const long P[3], const long Q[3], const long A[3], const long B[3], const long C[3]) {
  const int sp = sgn(orient_i(A, B, C, P)), sq = sgn(orient_i(A, B, C, Q));
  if (sp == 0 || sq == 0) return -1;
  if (sp == sq) return 0;
  const int s1 = sgn(orient_i(P, Q, A, B)), s2 = sgn(orient_i(P, Q, B, C)), s3 = sgn(orient_i(P, Q, C, A));
  if (s1 == 0 || s2 == 0 || s3 == 0) return -1;
  return (s1 == s2 && s2 == s3) ? 1 : 0;
}

/* 2-D: does segment PQ cross segment AB (coordinates u, v)? 1 / 0 / -1 degenerate */
static i128 orient2(const long a[2], const long b[2], const long c[2]) {
  return (i128)(b[0] - a[0]) * (c[1] - a[1]) - (i128)(b[1] - a[1]) * (c[0] - a[0]);
}
static int seg_seg(const long P[2], const long Q[2], const long A[2], const long B[2]) {
  const int a = sgn(orient2(P, Q, A)), b = sgn(orient2(P, Q, B));
  const int c = sgn(orient2(A, B, P)), d = sgn(orient2(A, B, Q));
  if (a == 0 || b == 0 || c == 0 || d == 0) return -1;
  return (a != b && c != d) ? 1 : 0;
}

static void lattice_pt(const float *Xg, int v, long out[3]) {
  for (int d = 0; d < 3; ++d) out[d] = (long)nearbyint(((double)Xg[3 * v + d] + 0.5) * 128.0);
}

static const long RAYS[6][3] = {{1L << 22, 1009, 2003}, {3001, 1L << 22, 4007}, {5003, 6007, 1L << 22},
                               {-(1L << 22), 7001, -8009}, {9001, -(1L << 22), 1013}, {-1019, 1021, -(1L << 22)}};

static int inside_link3(const ref_problem *p, const float *Xg, int v) {
  long P[3];
  lattice_pt(Xg, v, P);
  for (int r = 0; r < 6; ++r) {
    long Q[3] = {P[0] + RAYS[r][0], P[1] + RAYS[r][1], P[2] + RAYS[r][2]};
    int cross = 0, degenerate = 0;
    for (int j = p->star_off[v]; j < p->star_off[v + 1] && !degenerate; ++j) {
      const int *t = p->tet + 4 * p->star[j];
      long F[3][3];
      int m = 0;
      for (int q = 0; q < 4; ++q)
        if (t[q] != v) lattice_pt(Xg, t[q], F[m++]);
      const int hit = seg_tri(P, Q, F[0], F[1], F[2]);
      if (hit < 0)
        degenerate = 1;
      else
        cross += hit;
    }
    if (!degenerate) return cross & 1;
  }
  return 0; /* every direction degenerate: treated as a violation */
}

/* point on border plane `axis`: polygon of the in-plane edges opposite v */
static int inside_link2(const ref_problem *p, const float *Xg, int v, int axis) {
  const int ua = axis == 0 ? 1 : 0, va = axis == 2 ? 1 : 2;
  long P3[3];
  lattice_pt(Xg, v, P3);
  const long P[2] = {P3[ua], P3[va]};
  for (int r = 0; r < 6; ++r) {
    const long Q[2] = {P[0] + RAYS[r][0] + RAYS[r][2], P[1] + RAYS[r][1] - RAYS[r][2]};
    int cross = 0, degenerate = 0;
    for (int j = p->star_off[v]; j < p->star_off[v + 1] && !degenerate; ++j) {
      const int *t = p->tet + 4 * p->star[j];
      long E[2][3];
      int m = 0, on = 1;
      for (int q = 0; q < 4; ++q) {
        if (t[q] == v) continue;
        long w[3];
        lattice_pt(Xg, t[q], w);
        if (w[axis] != P3[axis]) {
          on = 0;
          continue;
        }
        if (m < 2) memcpy(E[m], w, sizeof(w));
        ++m;
      }
      if (!on && m != 2) continue; /* no border face with v in this tetrahedron */
      if (m != 2) continue;
      const long A[2] = {E[0][ua], E[0][va]}, B[2] = {E[1][ua], E[1][va]};
      const int hit = seg_seg(P, Q, A, B);
      if (hit < 0)
        degenerate = 1;
      else
        cross += hit;
    }
    if (!degenerate) return cross & 1;
  }
  return 0;
}

void ref_literal_fold_check(const ref_problem *p, int S, const float *X, int *violations) {
  for (int s = 0; s < S; ++s)
    for (int g = 0; g < 2; ++g) {
      const float *Xg = X + ((long)s * 2 + g) * p->P * 3;
      int bad = 0;
      for (int k = 0; k < p->n[2]; ++k)
        for (int j = 0; j < p->n[1]; ++j)
          for (int i = 0; i < p->n[0]; ++i) {
            const int v = pidx(p->n, i, j, k), idx[3] = {i, j, k};
            int nb = 0, axis = -1, free_axis = -1;
            for (int d = 0; d < 3; ++d) {
              if (idx[d] == 0 || idx[d] == p->n[d] - 1) {
                ++nb;
                axis = d;
              } else {
                free_axis = d;
              }
            }
            int ok = 1;
            if (nb == 0) {
              ok = inside_link3(p, Xg, v);
            } else if (nb == 1) {
              ok = inside_link2(p, Xg, v, axis);
            } else if (nb == 2) { /* border edge: strictly between its two neighbours on the edge */
              int lo[3] = {i, j, k}, hi[3] = {i, j, k};
              lo[free_axis] -= 1;
              hi[free_axis] += 1;
              const double x = Xg[3 * v + free_axis];
              ok = Xg[3 * pidx(p->n, lo[0], lo[1], lo[2]) + free_axis] < x &&
                   x < Xg[3 * pidx(p->n, hi[0], hi[1], hi[2]) + free_axis];
            }
            bad += !ok;
          }
      violations[s * 2 + g] = bad;
    }
}

/* threads the oracle's parallel loops use (timing legs); 0 leaves the default */
void ref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ref_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
