/*
 * sgrid_oracle.c -- plain, slow CPU oracle of the sparse-dense SDF grid
 * renderer of Dong et al., "Fast Monocular Scene Reconstruction with
 * Global-Sparse Local-Dense Grids" (CVPR 2023).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file; the product library never
 * does, and the two share no code.
 *
 * Precision.  The paper fixes none.  Where a floating-point value decides an
 * integer (which voxel and block a sample falls in, whether a lattice point
 * is inside [t_near, t_far]) the decision is taken in float32 with exactly
 * one rounding per operation -- build with -ffp-contract=off so that no
 * multiply-add is fused -- because that is the precision the GPU kernels
 * take it in.  Every other quantity (trilinear weights, SDF, gradient,
 * features, density, compositing, adjoint) is evaluated in double.
 *
 * Readings of the paper used here (each is also listed in the design notes):
 *  - voxel (i,j,k) sits at origin + (i,j,k)*h; block = floor(i/8); local
 *    index lx + 8 ly + 64 lz;
 *  - samples lie on the per-ray lattice t_k = t_near + k*step; a lattice
 *    point is kept iff the blocks of all 8 corners of its cell exist
 *    (sampling "in the sparse grid where valid blocks are allocated",
 *    Sec. 3.5.1); the first max_samples kept points are used;
 *  - delta_k = step for every kept sample (skipped space has no density);
 *  - density sigma = (1/beta) Psi_beta(-f), Psi_beta the zero-mean Laplace
 *    CDF with scale beta (VolSDF's transform named in Sec. 3.5.1);
 *  - depth is the ray distance t, the normal the raw gradient of Eq. 18,
 *    colour the raw interpolated features; no normalisation.
 *
 * Error codes: 0 ok, -1 bad argument, -2 coordinate out of range,
 * -3 out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define COORD_LIMIT 1048576 /* block coordinates lie in [-2^20, 2^20) */
#define VOX_PER_BLOCK 512
#define POS_LIMIT 16777216.0f /* |voxel-space position| beyond this: no block */

/* ------------------------------------------------------------------------ */
/* Block index: a sorted table of (packed coordinate, index), searched with
 * bsearch.  The plain definition of the hash of Sec. 3.2: a one-to-one map
 * from an allocated block coordinate to its index. */

typedef struct {
  int64_t key;
  int64_t pos; /* build: input position; lookup table: block index */
} entry;

static int64_t pack_key(int32_t x, int32_t y, int32_t z) {
  if (x < -COORD_LIMIT || x >= COORD_LIMIT || y < -COORD_LIMIT ||
      y >= COORD_LIMIT || z < -COORD_LIMIT || z >= COORD_LIMIT)
    return -1;
  return (((int64_t)x + COORD_LIMIT) << 42) | (((int64_t)y + COORD_LIMIT) << 21) |
         ((int64_t)z + COORD_LIMIT);
}

static int cmp_entry(const void* a, const void* b) {
  const entry* ea = (const entry*)a;
  const entry* eb = (const entry*)b;
  if (ea->key != eb->key) return ea->key < eb->key ? -1 : 1;
  if (ea->pos != eb->pos) return ea->pos < eb->pos ? -1 : 1;
  return 0;
}

static int cmp_key_only(const void* a, const void* b) {
  const entry* ea = (const entry*)a;
  const entry* eb = (const entry*)b;
  if (ea->key != eb->key) return ea->key < eb->key ? -1 : 1;
  return 0;
}

typedef struct {
  int64_t n;
  entry* e; /* sorted by key; pos = block index */
} table;

static int table_make(table* t, const int32_t* block_coords, int64_t n) {
  t->n = n;
  t->e = (entry*)malloc((size_t)(n > 0 ? n : 1) * sizeof(entry));
  if (!t->e) return -3;
  for (int64_t b = 0; b < n; ++b) {
    t->e[b].key = pack_key(block_coords[3 * b], block_coords[3 * b + 1],
                           block_coords[3 * b + 2]);
    if (t->e[b].key < 0) {
      free(t->e);
      return -2;
    }
    t->e[b].pos = b;
  }
  qsort(t->e, (size_t)n, sizeof(entry), cmp_entry);
  return 0;
}

static void table_free(table* t) { free(t->e); }

/* Index of block (x,y,z) or -1. */
static int64_t table_find(const table* t, int32_t x, int32_t y, int32_t z) {
  entry q;
  q.key = pack_key(x, y, z);
  if (q.key < 0) return -1;
  q.pos = 0;
  const entry* hit =
      (const entry*)bsearch(&q, t->e, (size_t)t->n, sizeof(entry), cmp_key_only);
  return hit ? hit->pos : -1;
}

/* floor(j / 8) for any int32 j. */
static int32_t floor_div8(int32_t j) {
  return (j >= 0) ? j / 8 : -((-j + 7) / 8);
}

static int32_t mod8(int32_t j) { return j - 8 * floor_div8(j); }

/*
 * Grid build: deduplicate block coordinates, index them in order of first
 * occurrence.  out_block_coords receives the unique coordinates in index
 * order ([n,3] capacity), out_index_of_input the index of every input row.
 */
int or_build(const int32_t* coords, int64_t n, int32_t* out_index_of_input,
             int32_t* out_block_coords, int64_t* out_n_blocks) {
  if (n < 0 || (n > 0 && (!coords || !out_block_coords)) || !out_n_blocks)
    return -1;
  entry* all = (entry*)malloc((size_t)(n > 0 ? n : 1) * sizeof(entry));
  if (!all) return -3;
  for (int64_t i = 0; i < n; ++i) {
    all[i].key = pack_key(coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]);
    if (all[i].key < 0) {
      free(all);
      return -2;
    }
    all[i].pos = i;
  }
  /* Sorting by (key, position) puts each group's first occurrence first. */
  qsort(all, (size_t)n, sizeof(entry), cmp_entry);
  /* first[i] = 1 iff input row i is the first occurrence of its key. */
  unsigned char* first = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  int64_t* group_first = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!first || !group_first) {
    free(all);
    free(first);
    free(group_first);
    return -3;
  }
  for (int64_t s = 0; s < n; ++s) {
    if (s == 0 || all[s].key != all[s - 1].key) first[all[s].pos] = 1;
  }
  /* Indices in input order of first occurrence. */
  int32_t* idx_of_pos = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!idx_of_pos) {
    free(all);
    free(first);
    free(group_first);
    return -3;
  }
  int64_t nb = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (first[i]) {
      idx_of_pos[i] = (int32_t)nb;
      out_block_coords[3 * nb] = coords[3 * i];
      out_block_coords[3 * nb + 1] = coords[3 * i + 1];
      out_block_coords[3 * nb + 2] = coords[3 * i + 2];
      ++nb;
    }
  }
  /* Every row takes the index of its group's first occurrence. */
  for (int64_t s = 0; s < n; ++s) {
    if (s == 0 || all[s].key != all[s - 1].key) group_first[s] = all[s].pos;
    else group_first[s] = group_first[s - 1];
    if (out_index_of_input)
      out_index_of_input[all[s].pos] = idx_of_pos[group_first[s]];
  }
  *out_n_blocks = nb;
  free(all);
  free(first);
  free(group_first);
  free(idx_of_pos);
  return 0;
}

/* Lookup of arbitrary coordinates against a block list (index order). */
int or_lookup(const int32_t* block_coords, int64_t n_blocks,
              const int32_t* query, int64_t m, int32_t* out_idx) {
  if (n_blocks < 0 || m < 0) return -1;
  table t;
  int rc = table_make(&t, block_coords, n_blocks);
  if (rc) return rc;
  for (int64_t i = 0; i < m; ++i)
    out_idx[i] = (int32_t)table_find(&t, query[3 * i], query[3 * i + 1], query[3 * i + 2]);
  table_free(&t);
  return 0;
}

/* Neighbour table: nbr[b][sx + 2 sy + 4 sz] = index of block b + (sx,sy,sz). */
int or_neighbors(const int32_t* block_coords, int64_t n_blocks, int32_t* out_nbr) {
  table t;
  int rc = table_make(&t, block_coords, n_blocks);
  if (rc) return rc;
  for (int64_t b = 0; b < n_blocks; ++b)
    for (int s = 0; s < 8; ++s)
      out_nbr[8 * b + s] = (int32_t)table_find(
          &t, block_coords[3 * b] + (s & 1), block_coords[3 * b + 1] + ((s >> 1) & 1),
          block_coords[3 * b + 2] + ((s >> 2) & 1));
  table_free(&t);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampling along a ray (Sec. 3.5.1): lattice t_k, fp32 positions, validity. */

typedef struct {
  float h, inv_h;      /* voxel size and its float32 reciprocal 1.0f/h */
  float org[3];        /* world position of voxel (0,0,0) */
  float step, t_near, t_far, beta;
  int32_t max_samples;
} geom;

typedef struct {
  int32_t k;       /* lattice index */
  float t;         /* t_k, float32 */
  int32_t i[3];    /* base voxel of the interpolation cell */
  float u[3];      /* position inside the cell, float32 */
  int64_t blk[8];  /* block of corner a = ax + 2 ay + 4 az */
  int32_t loc[8];  /* local index of that corner inside its block */
} sample;

/*
 * Locate voxel-space point (x,y,z) (float32): base voxel, fraction and the
 * 8 corner blocks.  Returns 1 iff all 8 corner blocks are allocated.
 */
static int locate(const table* tb, const float xv[3], sample* s) {
  for (int a = 0; a < 3; ++a) {
    if (!(fabsf(xv[a]) < POS_LIMIT)) return 0; /* also rejects NaN */
    float fl = floorf(xv[a]);
    s->i[a] = (int32_t)fl;
    s->u[a] = xv[a] - fl;
  }
  for (int a = 0; a < 8; ++a) {
    int32_t jx = s->i[0] + (a & 1);
    int32_t jy = s->i[1] + ((a >> 1) & 1);
    int32_t jz = s->i[2] + ((a >> 2) & 1);
    int64_t b = table_find(tb, floor_div8(jx), floor_div8(jy), floor_div8(jz));
    if (b < 0) return 0;
    s->blk[a] = b;
    s->loc[a] = mod8(jx) + 8 * mod8(jy) + 64 * mod8(jz);
  }
  return 1;
}

/*
 * All kept samples of one ray, in lattice order.  Returns their number
 * (<= g->max_samples).  Rays with a non-finite component keep none.
 */
static int ray_samples(const table* tb, const geom* g, const float ray[6], sample* out) {
  for (int a = 0; a < 6; ++a)
    if (!isfinite(ray[a])) return 0;
  float ov[3], dv[3];
  for (int a = 0; a < 3; ++a) {
    ov[a] = (ray[a] - g->org[a]) * g->inv_h;
    dv[a] = ray[3 + a] * g->inv_h;
  }
  int n = 0;
  for (int32_t k = 0; n < g->max_samples; ++k) {
    float t = g->t_near + (float)k * g->step;
    if (!(t <= g->t_far)) break;
    float xv[3];
    for (int a = 0; a < 3; ++a) {
      float td = t * dv[a];
      xv[a] = ov[a] + td;
    }
    sample s;
    if (locate(tb, xv, &s)) {
      s.k = k;
      s.t = t;
      out[n++] = s;
    }
  }
  return n;
}

static int geom_make(geom* g, float h, const float org[3], float step, float t_near,
                     float t_far, float beta, int32_t max_samples) {
  if (!(h > 0) || !isfinite(h) || !(step > 0) || !(beta > 0) || !isfinite(t_near) ||
      !isfinite(t_far) || max_samples < 1 || max_samples > 1024)
    return -1;
  if (!((t_far - t_near) / step < 16777216.0f)) return -1;
  g->h = h;
  g->inv_h = 1.0f / h;
  for (int a = 0; a < 3; ++a) g->org[a] = org[a];
  g->step = step;
  g->t_near = t_near;
  g->t_far = t_far;
  g->beta = beta;
  g->max_samples = max_samples;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Interpolation (Eq. 17-18) and density, in double. */

/* r_a and dr_a/du (per axis) for corner a at fraction u. */
static void corner_weights(const float uf[3], double r[8], double dr[8][3]) {
  double u[3] = {uf[0], uf[1], uf[2]};
  for (int a = 0; a < 8; ++a) {
    int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    double wx = ax ? u[0] : 1.0 - u[0];
    double wy = ay ? u[1] : 1.0 - u[1];
    double wz = az ? u[2] : 1.0 - u[2];
    r[a] = wx * wy * wz;
    dr[a][0] = (ax ? 1.0 : -1.0) * wy * wz;
    dr[a][1] = (ay ? 1.0 : -1.0) * wx * wz;
    dr[a][2] = (az ? 1.0 : -1.0) * wx * wy;
  }
}

/*
 * f, grad f (world units) and C features at a located sample.  The gradient
 * of Eq. 18, sum_a (dr_a/du) theta_a / h, is evaluated grouped by the edges
 * of the cell: d f/d u_x = sum over the 4 x-edges of (product of the other two
 * weights) * (theta at x=1 - theta at x=0), likewise for y and z.  This is
 * the same polynomial; grouping the two ends of each edge first makes a
 * direction in which the SDF is constant give exactly zero.
 */
/*
 * gmag (nullable): per axis, sum over the cell's edges along it of
 * |dr| (|theta_1| + |theta_0|) / h, the size of every term of the gradient
 * before the edge differences cancel: the scale of its float32 rounding.
 */
static void interpolate_mag(const sample* s, const double* vox, int C, double h,
                            double* f, double grad[3], double* feat, double gmag[3]) {
  double r[8], dr[8][3], th0[8];
  corner_weights(s->u, r, dr);
  *f = 0.0;
  for (int ch = 0; ch < C; ++ch) feat[ch] = 0.0;
  for (int a = 0; a < 8; ++a) {
    const double* th = vox + ((size_t)s->blk[a] * VOX_PER_BLOCK + (size_t)s->loc[a]) * (size_t)(1 + C);
    th0[a] = th[0];
    *f += r[a] * th[0];
    for (int ch = 0; ch < C; ++ch) feat[ch] += r[a] * th[1 + ch];
  }
  for (int ax = 0; ax < 3; ++ax) {
    const int bit = 1 << ax;
    double g = 0.0;
    double gm = 0.0;
    for (int a = 0; a < 8; ++a)
      if (!(a & bit)) {
        g += dr[a | bit][ax] * (th0[a | bit] - th0[a]); /* dr of the x=1 end: +w w */
        gm += fabs(dr[a | bit][ax]) * (fabs(th0[a | bit]) + fabs(th0[a]));
      }
    grad[ax] = g / h;
    if (gmag) gmag[ax] = gm / h;
  }
}

static void interpolate(const sample* s, const double* vox, int C, double h,
                        double* f, double grad[3], double* feat) {
  interpolate_mag(s, vox, C, h, f, grad, feat, NULL);
}

/* Laplace-CDF density sigma(f) = (1/beta) Psi_beta(-f) and d sigma / d f. */
static double density(double f, double beta, double* dsigma_df) {
  double s = -f, psi;
  if (s <= 0.0) psi = 0.5 * exp(s / beta);
  else psi = 1.0 - 0.5 * exp(-s / beta);
  if (dsigma_df) *dsigma_df = -exp(-fabs(f) / beta) / (2.0 * beta * beta);
  return psi / beta;
}

int or_density(const double* f, int64_t n, double beta, double* sigma, double* dsigma) {
  if (!(beta > 0)) return -1;
  for (int64_t i = 0; i < n; ++i) sigma[i] = density(f[i], beta, dsigma ? &dsigma[i] : NULL);
  return 0;
}

/* Point query (Eq. 17-18) at world points p [m,3]: valid flag, f, grad, feat. */
int or_query(const int32_t* block_coords, int64_t n_blocks, const double* vox, int32_t C,
             float h, const float org[3], const float* p, int64_t m, int32_t* valid,
             double* f, double* grad, double* feat) {
  if (C < 0 || !(h > 0)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  float inv_h = 1.0f / h;
  for (int64_t q = 0; q < m; ++q) {
    float xv[3];
    for (int a = 0; a < 3; ++a) xv[a] = (p[3 * q + a] - org[a]) * inv_h;
    sample s;
    valid[q] = locate(&tb, xv, &s);
    if (valid[q]) {
      interpolate(&s, vox, C, (double)h, &f[q], &grad[3 * q], C ? &feat[(size_t)C * q] : NULL);
    } else {
      f[q] = 0.0;
      grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = 0.0;
      for (int ch = 0; ch < C; ++ch) feat[(size_t)C * q + ch] = 0.0;
    }
  }
  table_free(&tb);
  return 0;
}

/*
 * Eikonal regulariser (Eq. 16) at points p [m,3], each with weight `weight`:
 * loss[q] = weight * (|g| - 1)^2 with g = grad f(p) of Eq. 18 (0 for points
 * that are not valid), and its derivative with respect to the SDF voxels.
 * g is linear in the SDF values, g = sum_a theta_a (dr_a/du) / h, so
 *   d loss / d theta_a = weight * 2 (|g| - 1) * (g / |g|) . (dr_a/du) / h.
 * The direction g / |g| is undefined at g = 0; the term is taken as 0 there.
 * grad_vox [n,512,1+C] is accumulated in channel 0.  Two scales for
 * tolerances: gmag [m] (nullable), the norm of the per-axis sums
 * sum_a |dr_a/du| |theta_a| / h (what bounds the rounding error of g), and
 * mag_vox [n,512] (nullable), which accumulates per term
 * 2 weight (|(|g| - 1)| + gmag) sum_axes |dr_a/du| / h, the size the term
 * can take when |g| moves by up to gmag (|g| - 1 cancels where |g| is near 1).
 */
/* The Eikonal term of one located sample: returns weight (|g| - 1)^2 and
 * accumulates its voxel gradient and scales (see or_eikonal). */
static double eik_sample(const sample* s, const double* vox, int C, double hd, double weight,
                         double* grad_vox, double* mag_vox, double* gmag) {
  double r[8], dr[8][3], th0[8];
  corner_weights(s->u, r, dr);
  for (int a = 0; a < 8; ++a)
    th0[a] = vox[((size_t)s->blk[a] * VOX_PER_BLOCK + (size_t)s->loc[a]) * (size_t)(1 + C)];
  /* g and its magnitude scale, from the plain sum over corners */
  double g[3], gm2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double acc = 0.0, am = 0.0;
    for (int a = 0; a < 8; ++a) {
      acc += dr[a][ax] * th0[a];
      am += fabs(dr[a][ax] * th0[a]);
    }
    g[ax] = acc / hd;
    gm2 += (am / hd) * (am / hd);
  }
  if (gmag) *gmag = sqrt(gm2);
  const double n = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (n > 0.0 && grad_vox) {
    const double coef = weight * 2.0 * (n - 1.0) / n;
    for (int a = 0; a < 8; ++a) {
      const size_t v = (size_t)s->blk[a] * VOX_PER_BLOCK + (size_t)s->loc[a];
      double t = 0.0, tm = 0.0;
      for (int ax = 0; ax < 3; ++ax) {
        t += coef * g[ax] * dr[a][ax] / hd;
        tm += 2.0 * fabs(weight) * (fabs(n - 1.0) + sqrt(gm2)) * fabs(dr[a][ax]) / hd;
      }
      grad_vox[v * (size_t)(1 + C)] += t;
      if (mag_vox) mag_vox[v] += tm;
    }
  }
  return weight * (n - 1.0) * (n - 1.0);
}

int or_eikonal(const int32_t* block_coords, int64_t n_blocks, const double* vox, int32_t C,
               float h, const float org[3], const float* p, int64_t m, double weight,
               double* loss, double* grad_vox, double* mag_vox, double* gmag) {
  if (C < 0 || !(h > 0)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  float inv_h = 1.0f / h;
  for (int64_t q = 0; q < m; ++q) {
    float xv[3];
    for (int a = 0; a < 3; ++a) xv[a] = (p[3 * q + a] - org[a]) * inv_h;
    sample s;
    loss[q] = 0.0;
    if (gmag) gmag[q] = 0.0;
    if (!locate(&tb, xv, &s)) continue;
    loss[q] = eik_sample(&s, vox, C, (double)h, weight, grad_vox, mag_vox, gmag ? &gmag[q] : NULL);
  }
  table_free(&tb);
  return 0;
}

/*
 * The Eikonal term on the ray samples of the render (the "ray-based samples
 * around surfaces" of Sec. 3.5.2): for each ray, loss_ray[r] = sum over its
 * kept samples (the samples the render uses, Sec. 3.5.1) of
 * weight * (|grad f(x_k)| - 1)^2, with the voxel gradient and scales of
 * or_eikonal accumulated over all samples.
 */
int or_eikonal_rays(const int32_t* block_coords, int64_t n_blocks, const double* vox, int32_t C,
                    float h, const float org[3], const float* rays, int64_t R, float step,
                    float t_near, float t_far, float beta, int32_t max_samples, double weight,
                    double* loss_ray, double* grad_vox, double* mag_vox) {
  if (C < 0 || R < 0) return -1;
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  sample* smp = (sample*)malloc((size_t)max_samples * sizeof(sample));
  if (!smp) {
    table_free(&tb);
    return -3;
  }
  for (int64_t r = 0; r < R; ++r) {
    int n = ray_samples(&tb, &g, rays + 6 * r, smp);
    double l = 0.0;
    for (int q = 0; q < n; ++q) l += eik_sample(&smp[q], vox, C, (double)h, weight, grad_vox, mag_vox, NULL);
    loss_ray[r] = l;
  }
  free(smp);
  table_free(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward render (Eq. 12-15). */

/*
 * For every ray: feat_out [R,C], depth [R], normal [R,3], wsum [R],
 * nsamples [R]; plus the magnitudes sum_k |w_k v_k| of every output element
 * (mag_* arrays, same shapes, nullable) used to scale tolerances; for the
 * normal, v_k is the sum of the absolute terms of the edge-grouped gradient
 * (before its edge differences cancel), so the scale bounds its rounding.
 */
int or_render_forward(const int32_t* block_coords, int64_t n_blocks, const double* vox,
                      int32_t C, float h, const float org[3], const float* rays, int64_t R,
                      float step, float t_near, float t_far, float beta, int32_t max_samples,
                      double* feat_out, double* depth, double* normal, double* wsum,
                      int32_t* nsamples, double* mag_feat, double* mag_depth,
                      double* mag_normal, double* mag_wsum) {
  if (C < 0 || C > 64 || R < 0) return -1;
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  sample* smp = (sample*)malloc((size_t)max_samples * sizeof(sample));
  double* c = (double*)malloc((size_t)(C > 0 ? C : 1) * sizeof(double));
  if (!smp || !c) {
    free(smp);
    free(c);
    table_free(&tb);
    return -3;
  }
  for (int64_t r = 0; r < R; ++r) {
    int n = ray_samples(&tb, &g, rays + 6 * r, smp);
    double accC[64], magC[64], accN[3] = {0, 0, 0}, magN[3] = {0, 0, 0};
    double accD = 0, magD = 0, accW = 0;
    for (int ch = 0; ch < C; ++ch) accC[ch] = magC[ch] = 0.0;
    double tau = 0.0; /* sum_{j<k} sigma_j delta_j */
    for (int q = 0; q < n; ++q) {
      double f, grad[3], gm[3];
      interpolate_mag(&smp[q], vox, C, (double)h, &f, grad, c, gm);
      double sigma = density(f, (double)beta, NULL);
      double T = exp(-tau);
      double alpha = -expm1(-sigma * (double)step); /* 1 - exp(-sigma delta) */
      double w = T * alpha;
      for (int ch = 0; ch < C; ++ch) {
        accC[ch] += w * c[ch];
        magC[ch] += fabs(w * c[ch]);
      }
      accD += w * (double)smp[q].t;
      magD += fabs(w * (double)smp[q].t);
      for (int a = 0; a < 3; ++a) {
        accN[a] += w * grad[a];
        magN[a] += fabs(w) * gm[a]; /* >= |w grad|: the terms before cancellation */
      }
      accW += w;
      tau += sigma * (double)step;
    }
    for (int ch = 0; ch < C; ++ch) {
      feat_out[(size_t)C * r + ch] = accC[ch];
      if (mag_feat) mag_feat[(size_t)C * r + ch] = magC[ch];
    }
    depth[r] = accD;
    for (int a = 0; a < 3; ++a) normal[3 * r + a] = accN[a];
    wsum[r] = accW;
    if (nsamples) nsamples[r] = n;
    if (mag_depth) mag_depth[r] = magD;
    if (mag_normal)
      for (int a = 0; a < 3; ++a) mag_normal[3 * r + a] = magN[a];
    if (mag_wsum) mag_wsum[r] = accW;
  }
  free(smp);
  free(c);
  table_free(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward: the adjoint of the forward render w.r.t. every voxel parameter. */

/*
 * Accumulates dL/dvox into grad_vox [n_blocks,512,1+C] for
 * L = sum_r g_feat.feat + g_depth depth + g_normal.normal + g_wsum wsum.
 * Derivation from Eq. 15: with s_k = dL/dw_k,
 *   dL/dsigma_k = delta (T_{k+1} s_k - sum_{j>k} w_j s_j),
 * T_{k+1} = exp(-sum_{j<=k} sigma_j delta); then through sigma(f) to the 8
 * corner SDF values (trilinear weights r_a), plus the normal term
 * w_k g_normal . grad_theta(grad f_k) (Eq. 18), and w_k r_a g_feat for the
 * features.  mag_vox (nullable) receives the sum of the absolute values of
 * every product term of that expansion, to scale tolerances.
 */
int or_render_backward(const int32_t* block_coords, int64_t n_blocks, const double* vox,
                       int32_t C, float h, const float org[3], const float* rays, int64_t R,
                       float step, float t_near, float t_far, float beta, int32_t max_samples,
                       const double* g_feat, const double* g_depth, const double* g_normal,
                       const double* g_wsum, double* grad_vox, double* mag_vox) {
  if (C < 0 || C > 64 || R < 0) return -1;
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  int M = max_samples;
  size_t Cc = (size_t)(C > 0 ? C : 1);
  sample* smp = (sample*)malloc((size_t)M * sizeof(sample));
  double* F = (double*)malloc((size_t)M * sizeof(double));
  double* G = (double*)malloc((size_t)M * 3 * sizeof(double));
  double* Cf = (double*)malloc((size_t)M * Cc * sizeof(double));
  double* SIG = (double*)malloc((size_t)M * sizeof(double));
  double* DSIG = (double*)malloc((size_t)M * sizeof(double));
  double* W = (double*)malloc((size_t)M * sizeof(double));
  double* TN = (double*)malloc((size_t)M * sizeof(double));
  double* S = (double*)malloc((size_t)M * sizeof(double));
  double* SA = (double*)malloc((size_t)M * sizeof(double));
  if (!smp || !F || !G || !Cf || !SIG || !DSIG || !W || !TN || !S || !SA) {
    rc = -3;
    goto done;
  }
  for (int64_t r = 0; r < R; ++r) {
    int n = ray_samples(&tb, &g, rays + 6 * r, smp);
    if (n == 0) continue;
    const double* gC = C ? g_feat + (size_t)C * r : NULL;
    double gD = g_depth[r];
    const double* gN = g_normal + 3 * r;
    double gW = g_wsum ? g_wsum[r] : 0.0;
    /* forward quantities */
    double tau = 0.0;
    for (int q = 0; q < n; ++q) {
      interpolate(&smp[q], vox, C, (double)h, &F[q], &G[3 * q], Cf + Cc * q);
      SIG[q] = density(F[q], (double)beta, &DSIG[q]);
      double T = exp(-tau);
      double alpha = -expm1(-SIG[q] * (double)step);
      W[q] = T * alpha;
      tau += SIG[q] * (double)step;
      TN[q] = exp(-tau); /* T_{k+1} */
      /* s_k = dL/dw_k, and its absolute-term counterpart */
      double s = gD * (double)smp[q].t + gW, sa = fabs(gD * (double)smp[q].t) + fabs(gW);
      for (int ch = 0; ch < C; ++ch) {
        s += gC[ch] * Cf[Cc * q + ch];
        sa += fabs(gC[ch] * Cf[Cc * q + ch]);
      }
      for (int a = 0; a < 3; ++a) {
        s += gN[a] * G[3 * q + a];
        sa += fabs(gN[a] * G[3 * q + a]);
      }
      S[q] = s;
      SA[q] = sa;
    }
    /* reverse pass: suffix sums sum_{j>k} w_j s_j */
    double suf = 0.0, sufa = 0.0;
    for (int q = n - 1; q >= 0; --q) {
      double dsig = (double)step * (TN[q] * S[q] - suf);
      double magsig = (double)step * (TN[q] * SA[q] + sufa);
      double df = dsig * DSIG[q];
      double magf = magsig * fabs(DSIG[q]);
      double rr[8], dr[8][3];
      corner_weights(smp[q].u, rr, dr);
      for (int a = 0; a < 8; ++a) {
        size_t base = ((size_t)smp[q].blk[a] * VOX_PER_BLOCK + (size_t)smp[q].loc[a]) * (size_t)(1 + C);
        double gn = 0.0, gna = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
          gn += dr[a][ax] * gN[ax];
          gna += fabs(dr[a][ax] * gN[ax]);
        }
        grad_vox[base] += rr[a] * df + W[q] * gn / (double)h;
        if (mag_vox) mag_vox[base] += rr[a] * magf + W[q] * gna / (double)h;
        for (int ch = 0; ch < C; ++ch) {
          grad_vox[base + 1 + ch] += W[q] * rr[a] * gC[ch];
          if (mag_vox) mag_vox[base + 1 + ch] += fabs(W[q] * rr[a] * gC[ch]);
        }
      }
      suf += W[q] * S[q];
      sufa += W[q] * SA[q];
    }
  }
  rc = 0;
done:
  free(smp);
  free(F);
  free(G);
  free(Cf);
  free(SIG);
  free(DSIG);
  free(W);
  free(TN);
  free(S);
  free(SA);
  table_free(&tb);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Sample lists and memory-footprint counts. */

/*
 * Kept samples of ray r (one ray): writes up to max_samples rows of
 * k, base voxel i[3], and the 8 corner block indices; returns the count
 * through *n_out.
 */
int or_ray_samples(const int32_t* block_coords, int64_t n_blocks, float h,
                   const float org[3], const float* ray, float step, float t_near,
                   float t_far, float beta, int32_t max_samples, int32_t* out_k,
                   float* out_t, int32_t* out_i, float* out_u, int64_t* out_blk,
                   int32_t* out_loc, int32_t* n_out) {
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  sample* smp = (sample*)malloc((size_t)max_samples * sizeof(sample));
  if (!smp) {
    table_free(&tb);
    return -3;
  }
  int n = ray_samples(&tb, &g, ray, smp);
  for (int q = 0; q < n; ++q) {
    out_k[q] = smp[q].k;
    out_t[q] = smp[q].t;
    for (int a = 0; a < 3; ++a) {
      out_i[3 * q + a] = smp[q].i[a];
      out_u[3 * q + a] = smp[q].u[a];
    }
    for (int a = 0; a < 8; ++a) {
      out_blk[8 * q + a] = smp[q].blk[a];
      out_loc[8 * q + a] = smp[q].loc[a];
    }
  }
  *n_out = n;
  free(smp);
  table_free(&tb);
  return 0;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int64_t count_distinct(int64_t* v, int64_t n) {
  if (n == 0) return 0;
  qsort(v, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t d = 1;
  for (int64_t i = 1; i < n; ++i)
    if (v[i] != v[i - 1]) ++d;
  return d;
}

/*
 * Per ray: S = kept samples, U = distinct voxels read (8 corners per sample),
 * K = distinct blocks holding them; counts [R,3].  touched (nullable,
 * uint8 [n_blocks*512]) is set to 1 for every voxel read by any ray.
 */
int or_render_footprint(const int32_t* block_coords, int64_t n_blocks, float h,
                        const float org[3], const float* rays, int64_t R, float step,
                        float t_near, float t_far, float beta, int32_t max_samples,
                        int32_t* counts, uint8_t* touched) {
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  sample* smp = (sample*)malloc((size_t)max_samples * sizeof(sample));
  int64_t* vox_ids = (int64_t*)malloc((size_t)max_samples * 8 * sizeof(int64_t));
  int64_t* blk_ids = (int64_t*)malloc((size_t)max_samples * 8 * sizeof(int64_t));
  if (!smp || !vox_ids || !blk_ids) {
    free(smp);
    free(vox_ids);
    free(blk_ids);
    table_free(&tb);
    return -3;
  }
  for (int64_t r = 0; r < R; ++r) {
    int n = ray_samples(&tb, &g, rays + 6 * r, smp);
    int64_t m = 0;
    for (int q = 0; q < n; ++q)
      for (int a = 0; a < 8; ++a) {
        vox_ids[m] = smp[q].blk[a] * VOX_PER_BLOCK + smp[q].loc[a];
        blk_ids[m] = smp[q].blk[a];
        if (touched) touched[vox_ids[m]] = 1;
        ++m;
      }
    counts[3 * r] = n;
    counts[3 * r + 1] = (int32_t)count_distinct(vox_ids, m);
    counts[3 * r + 2] = (int32_t)count_distinct(blk_ids, m);
  }
  free(smp);
  free(vox_ids);
  free(blk_ids);
  table_free(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Camera rays: inverse pinhole projection (the model of Eq. 3), in double. */

int or_rays_pinhole(const float* cams, int32_t n_cams, const int32_t* pix, int64_t R,
                    double* rays) {
  for (int64_t r = 0; r < R; ++r) {
    int32_t c = pix[3 * r];
    if (c < 0 || c >= n_cams) {
      for (int a = 0; a < 6; ++a) rays[6 * r + a] = NAN;
      continue;
    }
    const float* K = cams + 16 * (size_t)c;
    const float* M = K + 4; /* rows of [R | t] */
    double x = ((double)pix[3 * r + 1] + 0.5 - K[2]) / K[0];
    double y = ((double)pix[3 * r + 2] + 0.5 - K[3]) / K[1];
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = M[4 * a] * x + M[4 * a + 1] * y + M[4 * a + 2] * 1.0;
    double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) {
      rays[6 * r + a] = M[4 * a + 3];
      rays[6 * r + 3 + a] = d[a] / nrm;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Block allocation from depth (Sec. 3.4.1) and fusion (Sec. 3.4.2).         */

#define COORD_LIMIT 1048576 /* block coordinates lie in [-2^20, 2^20) */

typedef struct {
  uint64_t key;
  int64_t pos;
} keyed;

static int cmp_keyed(const void* a, const void* b) {
  const keyed* x = (const keyed*)a;
  const keyed* y = (const keyed*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->pos < y->pos ? -1 : (x->pos > y->pos);
}

static int cmp_pos(const void* a, const void* b) {
  const keyed* x = (const keyed*)a;
  const keyed* y = (const keyed*)b;
  return x->pos < y->pos ? -1 : (x->pos > y->pos);
}

static uint64_t coord_key(const int32_t* c) {
  return ((uint64_t)(uint32_t)(c[0] + COORD_LIMIT) << 42) |
         ((uint64_t)(uint32_t)(c[1] + COORD_LIMIT) << 21) | (uint64_t)(uint32_t)(c[2] + COORD_LIMIT);
}

/* Keep the first occurrence of every coordinate of c [n,3], in order; returns
 * the number kept (c is compacted in place), or -3 on allocation failure. */
static int64_t unique_first(int32_t* c, int64_t n) {
  if (n == 0) return 0;
  keyed* k = (keyed*)malloc((size_t)n * sizeof(keyed));
  if (!k) return -3;
  for (int64_t i = 0; i < n; ++i) {
    k[i].key = coord_key(c + 3 * i);
    k[i].pos = i;
  }
  qsort(k, (size_t)n, sizeof(keyed), cmp_keyed);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || k[i].key != k[i - 1].key) k[m++] = k[i];
  qsort(k, (size_t)m, sizeof(keyed), cmp_pos);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t p = k[i].pos; /* p >= i: copying forward is safe */
    c[3 * i] = c[3 * p];
    c[3 * i + 1] = c[3 * p + 1];
    c[3 * i + 2] = c[3 * p + 2];
  }
  free(k);
  return m;
}

/*
 * Blocks allocated from depth maps (Sec. 3.4.1): every pixel (u, v) of
 * frame f with a depth D (finite, 0 < D <= depth_max) is lifted to the
 * camera point (x D, y D, D), x = (u + 1/2 - cx) / fx, y = (v + 1/2 - cy) / fy
 * (the inverse projection of the pinhole model, depth along the optical
 * axis), moved to the world by [R | t], and its block floor(X / (8h)) taken
 * (through the voxel floor(X / h), as the march does); each such block is
 * dilated to the (2r+1)^3 blocks around it.  float32, one rounding per
 * operation, in the order written.  Output: the block coordinates in order of
 * first occurrence (frames, rows, columns, then dilation offsets z, y, x
 * from -r to r), duplicates removed.  cams [F,16] as in or_rays_pinhole;
 * depth [F,H,W].  Pixels whose blocks (dilated) would leave [-2^20, 2^20)
 * are skipped.  out [cap,3]; *n_out = number written; -2 if cap is too small.
 */
int or_alloc_blocks(const float* cams, int32_t F, const float* depth, int32_t W, int32_t H,
                    float h, const float org[3], int32_t r, float depth_max, int32_t* out,
                    int64_t cap, int64_t* n_out) {
  if (F < 0 || W < 0 || H < 0 || r < 0 || !(h > 0)) return -1;
  const float inv_h = 1.0f / h;
  const int64_t P = (int64_t)F * W * H;
  int32_t* b = (int32_t*)malloc((size_t)(P > 0 ? P : 1) * 3 * sizeof(int32_t));
  if (!b) return -3;
  int64_t nb = 0;
  for (int32_t f = 0; f < F; ++f) {
    const float* K = cams + 16 * (size_t)f;
    for (int32_t v = 0; v < H; ++v)
      for (int32_t u = 0; u < W; ++u) {
        const float D = depth[((size_t)f * H + v) * W + u];
        if (!(isfinite(D) && D > 0.0f && D <= depth_max)) continue;
        const float x = ((float)u + 0.5f - K[2]) / K[0];
        const float y = ((float)v + 0.5f - K[3]) / K[1];
        const float xc[3] = {x * D, y * D, D};
        int ok = 1;
        int32_t bb[3];
        for (int a = 0; a < 3; ++a) {
          const float* M = K + 4 + 4 * a;
          const float p0 = M[0] * xc[0];
          const float p1 = M[1] * xc[1];
          const float p2 = M[2] * xc[2];
          const float X = ((p0 + p1) + p2) + M[3];
          const float xv = (X - org[a]) * inv_h;
          if (!(fabsf(xv) < POS_LIMIT)) {
            ok = 0;
            break;
          }
          bb[a] = floor_div8((int32_t)floorf(xv));
          if (bb[a] - r < -COORD_LIMIT || bb[a] + r >= COORD_LIMIT) ok = 0;
        }
        if (!ok) continue;
        b[3 * nb] = bb[0];
        b[3 * nb + 1] = bb[1];
        b[3 * nb + 2] = bb[2];
        ++nb;
      }
  }
  int64_t nu = unique_first(b, nb);
  if (nu < 0) {
    free(b);
    return -3;
  }
  const int64_t side = 2 * (int64_t)r + 1, nd = nu * side * side * side;
  int32_t* d = (int32_t*)malloc((size_t)(nd > 0 ? nd : 1) * 3 * sizeof(int32_t));
  if (!d) {
    free(b);
    return -3;
  }
  int64_t m = 0;
  for (int64_t i = 0; i < nu; ++i)
    for (int32_t dz = -r; dz <= r; ++dz)
      for (int32_t dy = -r; dy <= r; ++dy)
        for (int32_t dx = -r; dx <= r; ++dx) {
          d[3 * m] = b[3 * i] + dx;
          d[3 * m + 1] = b[3 * i + 1] + dy;
          d[3 * m + 2] = b[3 * i + 2] + dz;
          ++m;
        }
  free(b);
  const int64_t no = unique_first(d, m);
  if (no < 0) {
    free(d);
    return -3;
  }
  *n_out = no;
  if (no > cap) {
    free(d);
    return -2;
  }
  memcpy(out, d, (size_t)no * 3 * sizeof(int32_t));
  free(d);
  return 0;
}

/*
 * Fusion (Sec. 3.4.2): every voxel v (world position origin + i h, float32)
 * is projected into every frame f: camera point c = R^T (X - t), pixel
 * (floor(fx c_x / c_z + cx), floor(fy c_y / c_z + cy)) (the pixel whose
 * centre ray the voxel is nearest to), and associated when c_z > 0, the
 * pixel lies in the image, its depth D is finite and > 0, and the voxel is
 * not more than trunc behind the surface (D - c_z >= -trunc; the truncation
 * of the supplement's Volumetric Fusion).  The least-squares solutions are
 * averages over the associations of the truncated projective SDF:
 *   vox[v,0]   = mean of min(D - c_z, trunc),
 *   vox[v,1+ch] = mean of feat[f,pixel,ch],
 * and the last n_sem feature channels (semantic logits) are divided by
 * their L2 norm.  A voxel with no association gets SDF = trunc and zero
 * features.  weight[v] = number of associations.  The decisions (pixel,
 * association) are taken in float32 in the order written, the averages in
 * double.  feat [F,H,W,C]; vox [n,512,1+C]; weight [n,512].
 */
int or_fuse(const int32_t* block_coords, int64_t n_blocks, float h, const float org[3],
            const float* cams, int32_t F, const float* depth, const float* feat, int32_t C,
            int32_t W, int32_t H, float trunc, int32_t n_sem, double* vox, double* weight) {
  if (n_blocks < 0 || F < 0 || C < 0 || n_sem < 0 || n_sem > C || !(h > 0) || !(trunc > 0))
    return -1;
  double* acc = (double*)malloc((size_t)(C > 0 ? C : 1) * sizeof(double));
  if (!acc) return -3;
  for (int64_t bi = 0; bi < n_blocks; ++bi)
    for (int l = 0; l < VOX_PER_BLOCK; ++l) {
      const int32_t li[3] = {l & 7, (l >> 3) & 7, l >> 6};
      float X[3];
      for (int a = 0; a < 3; ++a) {
        const float fi = (float)(8 * block_coords[3 * bi + a] + li[a]);
        const float step = fi * h;
        X[a] = org[a] + step;
      }
      double sd = 0.0;
      int64_t cnt = 0;
      for (int ch = 0; ch < C; ++ch) acc[ch] = 0.0;
      for (int32_t f = 0; f < F; ++f) {
        const float* K = cams + 16 * (size_t)f;
        float dd[3];
        for (int a = 0; a < 3; ++a) dd[a] = X[a] - K[4 + 4 * a + 3];
        float c[3];
        for (int j = 0; j < 3; ++j) {
          const float p0 = K[4 + j] * dd[0];     /* R[0][j] */
          const float p1 = K[8 + j] * dd[1];     /* R[1][j] */
          const float p2 = K[12 + j] * dd[2];    /* R[2][j] */
          c[j] = (p0 + p1) + p2;
        }
        const float z = c[2];
        if (!(z > 0.0f)) continue;
        const float qx = c[0] / z, qy = c[1] / z;
        const float uf = K[0] * qx + K[2];
        const float vf = K[1] * qy + K[3];
        if (!(uf >= 0.0f && uf < (float)W && vf >= 0.0f && vf < (float)H)) continue;
        const int32_t pu = (int32_t)floorf(uf), pv = (int32_t)floorf(vf);
        const size_t pix = ((size_t)f * H + pv) * W + pu;
        const float D = depth[pix];
        if (!(isfinite(D) && D > 0.0f)) continue;
        /* Truncation of the supplement's Volumetric Fusion: an association
           more than trunc behind the surface is rejected (occluded); in
           front of it the projective SDF is clipped to min(D - z, trunc). */
        const float s = D - z;
        if (!(s >= -trunc)) continue;
        {
          const double sdv = (double)D - (double)z;
          sd += sdv < (double)trunc ? sdv : (double)trunc;
        }
        for (int ch = 0; ch < C; ++ch) acc[ch] += feat[pix * C + ch];
        ++cnt;
      }
      double* o = vox + ((size_t)bi * VOX_PER_BLOCK + l) * (size_t)(1 + C);
      weight[(size_t)bi * VOX_PER_BLOCK + l] = (double)cnt;
      if (cnt == 0) {
        o[0] = trunc;
        for (int ch = 0; ch < C; ++ch) o[1 + ch] = 0.0;
        continue;
      }
      o[0] = sd / (double)cnt;
      for (int ch = 0; ch < C; ++ch) o[1 + ch] = acc[ch] / (double)cnt;
      if (n_sem > 0) {
        double nrm = 0.0;
        for (int ch = C - n_sem; ch < C; ++ch) nrm += o[1 + ch] * o[1 + ch];
        nrm = sqrt(nrm);
        for (int ch = C - n_sem; ch < C; ++ch) o[1 + ch] = nrm > 0.0 ? o[1 + ch] / nrm : 0.0;
      }
    }
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* De-noising (Sec. 3.4.3).                                                  */

/*
 * Gaussian blur of every property of every voxel over the allocated voxels
 * of its (2 radius + 1)^3 neighbourhood:
 *   out(v) = sum_d w(d) theta(v + d) / sum_d w(d),  w(d) = exp(-|d|^2 / (2 sigma^2)),
 * both sums over the offsets d whose voxel v + d lies in an allocated block
 * (the weights are renormalised where the neighbourhood leaves the grid).
 * vox, out [n,512,1+C]; mag (nullable) [n,512,1+C] receives
 * sum_d w(d) |theta(v + d)| / sum_d w(d) (the tolerance scale).
 */
int or_denoise(const int32_t* block_coords, int64_t n_blocks, const double* vox, int32_t C,
               int32_t radius, double sigma, double* out, double* mag) {
  if (n_blocks < 0 || C < 0 || radius < 0 || !(sigma > 0)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  const int V = 1 + C;
  for (int64_t b = 0; b < n_blocks; ++b)
    for (int l = 0; l < VOX_PER_BLOCK; ++l) {
      const int32_t gi[3] = {8 * block_coords[3 * b] + (l & 7), 8 * block_coords[3 * b + 1] + ((l >> 3) & 7),
                             8 * block_coords[3 * b + 2] + (l >> 6)};
      double* o = out + ((size_t)b * VOX_PER_BLOCK + l) * V;
      double* m = mag ? mag + ((size_t)b * VOX_PER_BLOCK + l) * V : NULL;
      double wsum = 0.0;
      for (int ch = 0; ch < V; ++ch) {
        o[ch] = 0.0;
        if (m) m[ch] = 0.0;
      }
      for (int dz = -radius; dz <= radius; ++dz)
        for (int dy = -radius; dy <= radius; ++dy)
          for (int dx = -radius; dx <= radius; ++dx) {
            const int32_t j[3] = {gi[0] + dx, gi[1] + dy, gi[2] + dz};
            const int64_t nb = table_find(&tb, floor_div8(j[0]), floor_div8(j[1]), floor_div8(j[2]));
            if (nb < 0) continue;
            const double w = exp(-(double)(dx * dx + dy * dy + dz * dz) / (2.0 * sigma * sigma));
            const double* th =
                vox + ((size_t)nb * VOX_PER_BLOCK + mod8(j[0]) + 8 * mod8(j[1]) + 64 * mod8(j[2])) * V;
            wsum += w;
            for (int ch = 0; ch < V; ++ch) {
              o[ch] += w * th[ch];
              if (m) m[ch] += w * fabs(th[ch]);
            }
          }
      for (int ch = 0; ch < V; ++ch) {
        o[ch] /= wsum; /* wsum > 0: the voxel itself is allocated */
        if (m) m[ch] /= wsum;
      }
    }
  table_free(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Permutohedral-lattice Gaussian filtering and a mean-field step of the     */
/* continuous CRF (Sec. 3.5.3).                                              */

#define LAT_MAX_D 24

/* Enclosing simplex of a d-dimensional (already scaled) feature position in
 * the permutohedral lattice A*_d: the position is lifted onto the plane
 * sum x = 0 of R^{d+1}, the nearest lattice point of remainder 0 is found
 * by rounding each coordinate to a multiple of d+1 and repairing the
 * coordinate sum through the ranks of the residuals; the d+1 vertices are
 * the remainder-0 point shifted by the canonical simplex of each remainder,
 * with barycentric weights from the sorted residuals.  float32, in the
 * order written (the vertices are integers decided in float32).
 * keys [(d+1) x d] (the first d coordinates of each vertex), w [d+1]. */
static void lattice_simplex(const float* pos, int d, int32_t* keys, double* w) {
  float el[LAT_MAX_D + 1];
  float sm = 0.0f;
  for (int i = d; i >= 1; --i) {
    const float scale = (float)(d + 1) * sqrtf(2.0f / 3.0f) / sqrtf((float)(i * (i + 1)));
    const float cf = pos[i - 1] * scale;
    el[i] = sm - (float)i * cf;
    sm += cf;
  }
  el[0] = sm;
  int32_t rem0[LAT_MAX_D + 1], rank[LAT_MAX_D + 1];
  int sum = 0;
  const float inv = 1.0f / (float)(d + 1);
  for (int i = 0; i <= d; ++i) {
    const float v = el[i] * inv;
    const float up = ceilf(v) * (float)(d + 1), dn = floorf(v) * (float)(d + 1);
    rem0[i] = (int32_t)((up - el[i] < el[i] - dn) ? up : dn);
    sum += rem0[i] / (d + 1);
    rank[i] = 0;
  }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j <= d; ++j) {
      const float di = el[i] - (float)rem0[i], dj = el[j] - (float)rem0[j];
      if (di < dj) ++rank[i];
      else ++rank[j];
    }
  for (int i = 0; i <= d; ++i) {
    if (sum > 0) {
      if (rank[i] >= d + 1 - sum) {
        rank[i] -= d + 1 - sum;
        rem0[i] -= d + 1;
      } else {
        rank[i] += sum;
      }
    } else if (sum < 0) {
      if (rank[i] < -sum) {
        rank[i] += d + 1 + sum;
        rem0[i] += d + 1;
      } else {
        rank[i] += sum;
      }
    }
  }
  double b[LAT_MAX_D + 2];
  for (int i = 0; i <= d + 1; ++i) b[i] = 0.0;
  for (int i = 0; i <= d; ++i) {
    const double t = ((double)el[i] - (double)rem0[i]) / (double)(d + 1);
    b[d - rank[i]] += t;
    b[d + 1 - rank[i]] -= t;
  }
  b[0] += 1.0 + b[d + 1];
  for (int r = 0; r <= d; ++r) {
    w[r] = b[r];
    for (int i = 0; i < d; ++i)
      keys[r * d + i] = rank[i] <= d - r ? rem0[i] + r : rem0[i] + r - (d + 1);
  }
}

typedef struct {
  int d, vd;
  int64_t cap, n;
  int32_t* keys; /* [cap][d] */
  uint8_t* used;
  double* val;   /* [cap][vd] */
} lattice;

static uint64_t lat_hash(const int32_t* k, int d) {
  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < d; ++i) {
    h ^= (uint64_t)(uint32_t)k[i];
    h *= 1099511628211ull;
  }
  return h;
}

/* index of key k, inserting it if absent and insert != 0; -1 if absent */
static int64_t lat_find(lattice* L, const int32_t* k, int insert) {
  uint64_t s = lat_hash(k, L->d) & (uint64_t)(L->cap - 1);
  for (;;) {
    if (!L->used[s]) {
      if (!insert) return -1;
      L->used[s] = 1;
      memcpy(L->keys + s * L->d, k, (size_t)L->d * sizeof(int32_t));
      ++L->n;
      return (int64_t)s;
    }
    if (memcmp(L->keys + s * L->d, k, (size_t)L->d * sizeof(int32_t)) == 0) return (int64_t)s;
    s = (s + 1) & (uint64_t)(L->cap - 1);
  }
}

/*
 * Gaussian filtering of values [N,vd] at feature positions pos [N,d]
 * (scaled so that the Gaussian has unit standard deviation per axis, as in
 * the permutohedral-lattice method the paper uses for the message passing):
 * splat each value onto the d+1 vertices of its simplex with its
 * barycentric weights, blur the lattice along each of its d+1 directions
 * with the [1/4, 1/2, 1/4] kernel (missing neighbours count as zero), and
 * slice back with the same weights.  out [N,vd] is that (unnormalised)
 * filter response; n_vertices (nullable) the number of lattice points.
 * Returns -1 for bad sizes, -3 if out of memory.
 */
static int lattice_filter_dirs(const float* pos, int64_t N, int32_t d, const double* val,
                               int32_t vd, double* out, int64_t* n_vertices, int reverse) {
  if (d < 1 || d > LAT_MAX_D || vd < 1 || N < 0) return -1;
  lattice L;
  L.d = d;
  L.vd = vd;
  L.n = 0;
  L.cap = 1;
  while (L.cap < 2 * (N * (d + 1) + 1)) L.cap <<= 1;
  L.keys = (int32_t*)malloc((size_t)L.cap * d * sizeof(int32_t));
  L.used = (uint8_t*)calloc((size_t)L.cap, 1);
  L.val = (double*)calloc((size_t)L.cap * vd, sizeof(double));
  double* tmp = (double*)calloc((size_t)L.cap * vd, sizeof(double));
  int64_t* vid = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * (d + 1) * sizeof(int64_t));
  double* bw = (double*)malloc((size_t)(N > 0 ? N : 1) * (d + 1) * sizeof(double));
  if (!L.keys || !L.used || !L.val || !tmp || !vid || !bw) {
    free(L.keys); free(L.used); free(L.val); free(tmp); free(vid); free(bw);
    return -3;
  }
  int32_t keys[(LAT_MAX_D + 1) * LAT_MAX_D];
  double w[LAT_MAX_D + 1];
  for (int64_t i = 0; i < N; ++i) { /* splat */
    lattice_simplex(pos + i * d, d, keys, w);
    for (int r = 0; r <= d; ++r) {
      const int64_t s = lat_find(&L, keys + r * d, 1);
      vid[i * (d + 1) + r] = s;
      bw[i * (d + 1) + r] = w[r];
      for (int c = 0; c < vd; ++c) L.val[s * vd + c] += w[r] * val[i * vd + c];
    }
  }
  int32_t nk[LAT_MAX_D];
  for (int jj = 0; jj <= d; ++jj) { /* blur along direction j */
    const int j = reverse ? d - jj : jj;
    for (int64_t s = 0; s < L.cap; ++s) {
      if (!L.used[s]) continue;
      const int32_t* k = L.keys + s * d;
      double* o = tmp + s * vd;
      for (int c = 0; c < vd; ++c) o[c] = 0.5 * L.val[s * vd + c];
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        /* neighbour: +/- ((1,...,1) - (d+1) e_j), first d coordinates */
        for (int i = 0; i < d; ++i) nk[i] = k[i] + sgn * (i == j ? -d : 1);
        const int64_t t = lat_find(&L, nk, 0);
        if (t < 0) continue;
        for (int c = 0; c < vd; ++c) o[c] += 0.25 * L.val[t * vd + c];
      }
    }
    double* sw = L.val;
    L.val = tmp;
    tmp = sw;
  }
  for (int64_t i = 0; i < N; ++i) /* slice */
    for (int c = 0; c < vd; ++c) {
      double acc = 0.0;
      for (int r = 0; r <= d; ++r) acc += bw[i * (d + 1) + r] * L.val[vid[i * (d + 1) + r] * vd + c];
      out[i * vd + c] = acc;
    }
  if (n_vertices) *n_vertices = L.n;
  free(L.keys); free(L.used); free(L.val); free(tmp); free(vid); free(bw);
  return 0;
}

int or_lattice_filter(const float* pos, int64_t N, int32_t d, const double* val, int32_t vd,
                      double* out, int64_t* n_vertices) {
  return lattice_filter_dirs(pos, N, d, val, vd, out, n_vertices, 0);
}

/*
 * Adjoint (transpose) of the lattice filter: the filter is slice . B_d ...
 * B_0 . splat with slice the transpose of splat and every single-direction
 * blur B_j symmetric (a neighbour pair exists from both ends), so its
 * transpose is the same splat and slice around the blurs in the reverse
 * direction order.
 */
int or_lattice_filter_adjoint(const float* pos, int64_t N, int32_t d, const double* val,
                              int32_t vd, double* out) {
  return lattice_filter_dirs(pos, N, d, val, vd, out, NULL, 1);
}

/* The simplex of each position (see lattice_simplex): keys [N][d+1][d],
 * weights [N][d+1]. */
int or_lattice_simplex(const float* pos, int64_t N, int32_t d, int32_t* keys, double* w) {
  if (d < 1 || d > LAT_MAX_D || N < 0) return -1;
  for (int64_t i = 0; i < N; ++i)
    lattice_simplex(pos + i * d, d, keys + i * (int64_t)(d + 1) * d, w + i * (d + 1));
  return 0;
}

/*
 * Mean-field inference of the CRF's label distribution (Sec. 3.5.3, after
 * Krahenbuhl and Koltun): Q = softmax(-unary), then T times
 *   Q(x_i) <- softmax_l( -unary_i(l) + w_p * m_i(l) ),  m = lattice filter of Q,
 * the update of the mean-field equation with a Potts compatibility of
 * weight w_p (the sum over the other labels differs from -m_i(l) by a
 * per-point constant, which the softmax removes).  The message includes
 * each point's own contribution.  unary, Q [N,L].
 */
int or_crf_meanfield(const float* pos, int64_t N, int32_t d, const double* unary, int32_t L,
                     double w_p, int32_t T, double* Q) {
  if (L < 1 || T < 0) return -1;
  double* m = (double*)malloc((size_t)(N > 0 ? N : 1) * L * sizeof(double));
  if (!m) return -3;
  for (int64_t i = 0; i < N; ++i) {
    double mx = -INFINITY, s = 0.0;
    for (int l = 0; l < L; ++l) mx = fmax(mx, -unary[i * L + l]);
    for (int l = 0; l < L; ++l) s += exp(-unary[i * L + l] - mx);
    for (int l = 0; l < L; ++l) Q[i * L + l] = exp(-unary[i * L + l] - mx) / s;
  }
  for (int it = 0; it < T; ++it) {
    int rc = or_lattice_filter(pos, N, d, Q, L, m, NULL);
    if (rc) {
      free(m);
      return rc;
    }
    for (int64_t i = 0; i < N; ++i) {
      double mx = -INFINITY, s = 0.0;
      for (int l = 0; l < L; ++l) mx = fmax(mx, -unary[i * L + l] + w_p * m[i * L + l]);
      for (int l = 0; l < L; ++l) s += exp(-unary[i * L + l] + w_p * m[i * L + l] - mx);
      for (int l = 0; l < L; ++l) Q[i * L + l] = exp(-unary[i * L + l] + w_p * m[i * L + l] - mx) / s;
    }
  }
  free(m);
  return 0;
}

/*
 * Mean-field inference with a general label compatibility (Sec. 3.5.3: the
 * pairwise potential is a compatibility mu(l, l') times the Gaussian
 * kernel of the feature distance).  Q = softmax(-unary), then T times
 *   Q_i(l) <- softmax_l( -unary_i(l) - sum_l' mu[l][l'] m_i(l') ),
 *   m = lattice filter of Q (each point's own contribution included).
 * compat [L,L] row-major: row l holds mu(l, .).  The Potts model is
 * mu = w (1 - I).  unary, Q [N,L].
 */
int or_crf_meanfield_compat(const float* pos, int64_t N, int32_t d, const double* unary,
                            int32_t L, const double* compat, int32_t T, double* Q) {
  if (L < 1 || T < 0) return -1;
  const size_t nl = (size_t)(N > 0 ? N : 1) * L;
  double* m = (double*)malloc(nl * sizeof(double));
  double* a = (double*)malloc((size_t)L * sizeof(double));
  if (!m || !a) {
    free(m);
    free(a);
    return -3;
  }
  for (int it = 0; it <= T; ++it) {
    if (it > 0) {
      int rc = or_lattice_filter(pos, N, d, Q, L, m, NULL);
      if (rc) {
        free(m);
        free(a);
        return rc;
      }
    }
    for (int64_t i = 0; i < N; ++i) {
      double mx = -INFINITY, s = 0.0;
      for (int l = 0; l < L; ++l) {
        double e = -unary[i * L + l];
        if (it > 0)
          for (int k = 0; k < L; ++k) e -= compat[l * L + k] * m[i * L + k];
        a[l] = e;
        mx = fmax(mx, e);
      }
      for (int l = 0; l < L; ++l) {
        a[l] = exp(a[l] - mx);
        s += a[l];
      }
      for (int l = 0; l < L; ++l) Q[i * L + l] = a[l] / s;
    }
  }
  free(m);
  free(a);
  return 0;
}

/*
 * Gradient of or_crf_meanfield_compat: for upstream gQ = dE/dQ [N,L] of the
 * final marginals of a scalar E, writes g_unary = dE/dunary [N,L] and
 * g_compat = dE/dmu [L,L].  Reverse mode through the T updates, each
 * Q = softmax(a), a = -unary - m mu^T, m = F(Q_prev):
 *   ga = Q * (gQ - <Q, gQ>)          (softmax adjoint, per point)
 *   g_unary -= ga;  g_compat(l,k) -= sum_i ga_i(l) m_i(k);
 *   gm_i(k) = -sum_l ga_i(l) mu(l,k);  gQ_prev = F^T(gm),
 * and finally g_unary -= ga of Q_0 = softmax(-unary).  The marginals of
 * every update are recomputed and kept.
 */
int or_crf_meanfield_compat_backward(const float* pos, int64_t N, int32_t d, const double* unary,
                                     int32_t L, const double* compat, int32_t T, const double* gQ,
                                     double* g_unary, double* g_compat) {
  if (L < 1 || T < 0 || N < 0) return -1;
  const size_t nl = (size_t)(N > 0 ? N : 1) * L;
  double* Qs = (double*)malloc(nl * (size_t)(T + 1) * sizeof(double));
  double* m = (double*)malloc(nl * sizeof(double));
  double* g = (double*)malloc(nl * sizeof(double));
  double* gm = (double*)malloc(nl * sizeof(double));
  double* ga = (double*)malloc((size_t)L * sizeof(double));
  int rc = 0;
  if (!Qs || !m || !g || !gm || !ga) {
    rc = -3;
    goto done;
  }
  for (int t = 0; t <= T; ++t) { /* forward, keeping every Q_t */
    rc = or_crf_meanfield_compat(pos, N, d, unary, L, compat, t, Qs + (size_t)t * nl);
    if (rc) goto done;
  }
  for (size_t e = 0; e < (size_t)N * L; ++e) {
    g_unary[e] = 0.0;
    g[e] = gQ[e];
  }
  for (int e = 0; e < L * L; ++e) g_compat[e] = 0.0;
  for (int t = T; t >= 0; --t) {
    const double* Q = Qs + (size_t)t * nl;
    if (t > 0) {
      rc = or_lattice_filter(pos, N, d, Qs + (size_t)(t - 1) * nl, L, m, NULL);
      if (rc) goto done;
    }
    for (int64_t i = 0; i < N; ++i) {
      double dot = 0.0;
      for (int l = 0; l < L; ++l) dot += Q[i * L + l] * g[i * L + l];
      for (int l = 0; l < L; ++l) {
        ga[l] = Q[i * L + l] * (g[i * L + l] - dot);
        g_unary[i * L + l] -= ga[l];
      }
      if (t == 0) continue;
      for (int l = 0; l < L; ++l)
        for (int k = 0; k < L; ++k) g_compat[l * L + k] -= ga[l] * m[i * L + k];
      for (int k = 0; k < L; ++k) {
        double acc = 0.0;
        for (int l = 0; l < L; ++l) acc -= ga[l] * compat[l * L + k];
        gm[i * L + k] = acc;
      }
    }
    if (t > 0) {
      rc = or_lattice_filter_adjoint(pos, N, d, gm, L, g);
      if (rc) goto done;
    }
  }
done:
  free(Qs);
  free(m);
  free(g);
  free(gm);
  free(ga);
  return rc;
}

/*
 * Adjoint of the point query (Eq. 17-18) with respect to the voxels: for
 * upstream gradients g_f [m], g_grad [m,3], g_feat [m,C] (each nullable) of
 * a scalar loss, accumulates into grad_vox [n,512,1+C]
 *   channel 0:   r_a g_f + (dr_a/du . g_grad) / h
 *   channel 1+c: r_a g_feat[c]
 * for the 8 corners a of every valid point; mag_vox (nullable, same shape)
 * accumulates the absolute values of the terms.
 */
int or_query_backward(const int32_t* block_coords, int64_t n_blocks, int32_t C, float h,
                      const float org[3], const float* p, int64_t m, const double* g_f,
                      const double* g_grad, const double* g_feat, double* grad_vox,
                      double* mag_vox) {
  if (C < 0 || !(h > 0)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  const float inv_h = 1.0f / h;
  const size_t V = (size_t)(1 + C);
  for (int64_t q = 0; q < m; ++q) {
    float xv[3];
    for (int a = 0; a < 3; ++a) xv[a] = (p[3 * q + a] - org[a]) * inv_h;
    sample s;
    if (!locate(&tb, xv, &s)) continue;
    double r[8], dr[8][3];
    corner_weights(s.u, r, dr);
    for (int a = 0; a < 8; ++a) {
      const size_t v = ((size_t)s.blk[a] * VOX_PER_BLOCK + (size_t)s.loc[a]) * V;
      double t0 = 0.0, m0 = 0.0;
      if (g_f) {
        t0 += r[a] * g_f[q];
        m0 += fabs(r[a] * g_f[q]);
      }
      if (g_grad)
        for (int ax = 0; ax < 3; ++ax) {
          t0 += dr[a][ax] * g_grad[3 * q + ax] / (double)h;
          m0 += fabs(dr[a][ax] * g_grad[3 * q + ax] / (double)h);
        }
      grad_vox[v] += t0;
      if (mag_vox) mag_vox[v] += m0;
      if (g_feat)
        for (int c = 0; c < C; ++c) {
          grad_vox[v + 1 + c] += r[a] * g_feat[(size_t)C * q + c];
          if (mag_vox) mag_vox[v + 1 + c] += fabs(r[a] * g_feat[(size_t)C * q + c]);
        }
    }
  }
  table_free(&tb);
  return 0;
}

/*
 * Label loss of the continuous CRF (Sec. 3.5.3, Eq. 22), the f-divergence
 * taken as the Kullback-Leibler divergence: for each node, x = softmax of
 * its label logits [L] and Q its mean-field marginals (a fixed target),
 *   loss[i] = weight * sum_l x_l log(x_l / Q_l),
 *   g[i,k]  = d loss[i] / d logit_k = weight * x_k (a_k - sum_l x_l a_l),
 *             a_l = log x_l - log Q_l.
 */
int or_crf_label_loss(const double* logits, const double* Q, int64_t N, int32_t L, double weight,
                      double* loss, double* g) {
  if (L < 1 || N < 0) return -1;
  for (int64_t i = 0; i < N; ++i) {
    const double* s = logits + i * L;
    double mx = -INFINITY, z = 0.0;
    for (int l = 0; l < L; ++l) mx = fmax(mx, s[l]);
    for (int l = 0; l < L; ++l) z += exp(s[l] - mx);
    double kl = 0.0;
    for (int l = 0; l < L; ++l) {
      const double lx = s[l] - mx - log(z);
      kl += exp(lx) * (lx - log(Q[i * L + l]));
    }
    loss[i] = weight * kl;
    for (int k = 0; k < L; ++k) {
      const double lx = s[k] - mx - log(z);
      g[i * L + k] = weight * exp(lx) * ((lx - log(Q[i * L + k])) - kl);
    }
  }
  return 0;
}

/*
 * Colour / normal loss of the continuous CRF (Sec. 3.5.3, Eq. 22) for a
 * continuous property x [n,P]: its mean-field estimate is the normalised
 * Gaussian filter of the property over the other features,
 * Q_i = F(x)_i / F(1)_i (filt [n,P+1] holds F applied to [x, 1]), a fixed
 * target; loss[i] = weight |x_i - Q_i|^2, g[i] = 2 weight (x_i - Q_i).
 */
int or_crf_property_loss(const double* x, const double* filt, int64_t N, int32_t P,
                         double weight, double* loss, double* g) {
  if (P < 1 || N < 0) return -1;
  for (int64_t i = 0; i < N; ++i) {
    const double den = filt[i * (P + 1) + P];
    double l = 0.0;
    for (int k = 0; k < P; ++k) {
      const double q = filt[i * (P + 1) + k] / den;
      const double d = x[i * P + k] - q;
      l += d * d;
      g[i * P + k] = 2.0 * weight * d;
    }
    loss[i] = weight * l;
  }
  return 0;
}

/*
 * Surface points of rays (the nodes of the continuous CRF are zero
 * crossings of the SDF seen from random viewpoints, Sec. 3.5.3): along the
 * kept samples of each ray (Sec. 3.5.1), the first pair of lattice-adjacent
 * samples with f_j > 0 >= f_{j+1} (entering the surface); the crossing is
 * placed by linear interpolation of f, t* = t_j + step f_j / (f_j - f_{j+1}),
 * at o + t* d.  hit [R] (1 / 0), points [R,3] (0 where no hit), and
 * margin [R] (nullable) = min(|f_j|, |f_{j+1}|) of the pair (how far the
 * sign decisions are from zero).
 */
int or_surface_points(const int32_t* block_coords, int64_t n_blocks, const double* vox, int32_t C,
                      float h, const float org[3], const float* rays, int64_t R, float step,
                      float t_near, float t_far, float beta, int32_t max_samples, int32_t* hit,
                      double* points, double* margin) {
  if (C < 0 || R < 0) return -1;
  geom g;
  if (geom_make(&g, h, org, step, t_near, t_far, beta, max_samples)) return -1;
  table tb;
  int rc = table_make(&tb, block_coords, n_blocks);
  if (rc) return rc;
  sample* smp = (sample*)malloc((size_t)max_samples * sizeof(sample));
  double* f = (double*)malloc((size_t)max_samples * sizeof(double));
  double* feat = (double*)malloc((size_t)(C > 0 ? C : 1) * sizeof(double));
  if (!smp || !f || !feat) {
    free(smp); free(f); free(feat);
    table_free(&tb);
    return -3;
  }
  for (int64_t r = 0; r < R; ++r) {
    const int n = ray_samples(&tb, &g, rays + 6 * r, smp);
    for (int j = 0; j < n; ++j) {
      double gr[3];
      interpolate(&smp[j], vox, C, (double)h, &f[j], gr, feat);
    }
    hit[r] = 0;
    points[3 * r] = points[3 * r + 1] = points[3 * r + 2] = 0.0;
    if (margin) margin[r] = 0.0;
    for (int j = 0; j + 1 < n; ++j) {
      if (smp[j + 1].k != smp[j].k + 1) continue;
      if (!(f[j] > 0.0 && f[j + 1] <= 0.0)) continue;
      const double ts = (double)smp[j].t + (double)step * f[j] / (f[j] - f[j + 1]);
      for (int a = 0; a < 3; ++a) points[3 * r + a] = (double)rays[6 * r + a] + ts * (double)rays[6 * r + 3 + a];
      hit[r] = 1;
      if (margin) margin[r] = fmin(fabs(f[j]), fabs(f[j + 1]));
      break;
    }
  }
  free(smp); free(f); free(feat);
  table_free(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Uniform samples in the sparse grid (the Eikonal term's "uniform samples  */
/* in the sparse grids", Sec. 3.5.2).                                        */

/* SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator:
 * output for counter c = the mix of c + 0x9e3779b97f4a7c15. */
uint64_t or_splitmix64(uint64_t c) {
  uint64_t z = c + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/*
 * n points uniform over the allocated blocks: point i draws x_k =
 * splitmix64(seed + 4 i + k), k = 0..3; block = x_0 mod n_blocks, and
 * u_a = (x_{1+a} >> 40) 2^-24 in [0,1) places it in the block: voxel
 * coordinate v_a = 8 b_a + 8 u_a, world position origin_a + v_a h (float32,
 * one rounding per operation in this order).  out [n,3].
 */
int or_uniform_points(const int32_t* block_coords, int64_t n_blocks, float h, const float org[3],
                      int64_t n, uint64_t seed, float* out) {
  if (n_blocks < 1 || n < 0 || !(h > 0)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t base = seed + 4ull * (uint64_t)i;
    const int64_t b = (int64_t)(or_splitmix64(base) % (uint64_t)n_blocks);
    for (int a = 0; a < 3; ++a) {
      const float u = (float)(or_splitmix64(base + 1 + a) >> 40) * 5.9604644775390625e-8f; /* 2^-24 */
      const float v0 = (float)(8 * block_coords[3 * b + a]);
      const float v = v0 + 8.0f * u;
      const float d = v * h;
      out[3 * i + a] = org[a] + d;
    }
  }
  return 0;
}
