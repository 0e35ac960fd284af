/*
 * Synthetic LiDAR scan simulator (test and benchmark input generation only).
 *
 * Casts rays from a sensor origin against a scene made of spheres, axis-aligned
 * boxes and capsules, and returns the first hit of each ray, perturbed along the
 * ray by Gaussian range noise.  Ray directions follow a 2-D Halton sequence over
 * (azimuth, elevation) whose index continues from frame to frame, which gives
 * the sparse, non-repetitive coverage of a Livox Mid-360 style scanner (the
 * paper approximates that sensor with a Halton ray pattern in its synthetic
 * evaluation, Section 4.1).
 *
 * Nothing here computes any part of the accessibility method: it only produces
 * the point clouds that both the oracle and the GPU library consume.
 *
 * Random numbers come from a counter-based generator (SplitMix64 finaliser of a
 * per-ray counter), so a frame is a pure function of (seed, frame, ray index)
 * and does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double a[3], b[3], r;
} capsule_t;

typedef struct {
  int ncap, nsph, nbox;
  capsule_t *cap;
  double *sph; /* nsph x 4: cx cy cz r */
  double *box; /* nbox x 6: lox loy loz hix hiy hiz */
  /* uniform grid over the capsules */
  double lo[3], cell;
  int dim[3];
  int *cell_start; /* dim0*dim1*dim2 + 1 */
  int *cell_items;
} scene_t;

static inline double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Smallest root t > tmin of |o + t d - c|^2 = r^2 (d unit), or INFINITY. */
static double hit_sphere(const double *o, const double *d, const double *c,
                         double r, double tmin) {
  double oc[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
  double b = dot3(oc, d);
  double cc = dot3(oc, oc) - r * r;
  double h = b * b - cc;
  if (h < 0) return INFINITY;
  h = sqrt(h);
  double t0 = -b - h, t1 = -b + h;
  if (t0 > tmin) return t0;
  if (t1 > tmin) return t1;
  return INFINITY;
}

/* Slab test; entry distance if > tmin. */
static double hit_box(const double *o, const double *d, const double *bx,
                      double tmin) {
  double t0 = -INFINITY, t1 = INFINITY;
  for (int i = 0; i < 3; ++i) {
    if (d[i] == 0.0) {
      if (o[i] < bx[i] || o[i] > bx[3 + i]) return INFINITY;
      continue;
    }
    double inv = 1.0 / d[i];
    double ta = (bx[i] - o[i]) * inv, tb = (bx[3 + i] - o[i]) * inv;
    if (ta > tb) {
      double t = ta;
      ta = tb;
      tb = t;
    }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
  }
  if (t0 > t1) return INFINITY;
  if (t0 > tmin) return t0;
  return INFINITY;
}

/* Capsule = points within r of segment [a,b]: the side of the infinite
 * cylinder restricted to the segment's span, plus the two end spheres. */
static double hit_capsule(const double *o, const double *d, const capsule_t *c,
                          double tmin) {
  double best = INFINITY;
  double ax[3] = {c->b[0] - c->a[0], c->b[1] - c->a[1], c->b[2] - c->a[2]};
  double len2 = dot3(ax, ax);
  double oa[3] = {o[0] - c->a[0], o[1] - c->a[1], o[2] - c->a[2]};
  if (len2 > 0) {
    double dd = dot3(d, ax), od = dot3(oa, ax);
    /* components perpendicular to the axis */
    double dp[3], op[3];
    for (int i = 0; i < 3; ++i) {
      dp[i] = d[i] - ax[i] * (dd / len2);
      op[i] = oa[i] - ax[i] * (od / len2);
    }
    double A = dot3(dp, dp), B = dot3(op, dp), C = dot3(op, op) - c->r * c->r;
    if (A > 1e-18) {
      double h = B * B - A * C;
      if (h >= 0) {
        h = sqrt(h);
        double ts[2] = {(-B - h) / A, (-B + h) / A};
        for (int k = 0; k < 2; ++k) {
          double t = ts[k];
          if (t <= tmin || t >= best) continue;
          double s = (od + t * dd) / len2;
          if (s >= 0.0 && s <= 1.0) best = t;
        }
      }
    }
  }
  double t = hit_sphere(o, d, c->a, c->r, tmin);
  if (t < best) best = t;
  t = hit_sphere(o, d, c->b, c->r, tmin);
  if (t < best) best = t;
  return best;
}

static inline int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

void *rc_create(const double *caps, int ncap, const double *sph, int nsph,
                const double *box, int nbox, double cell) {
  scene_t *s = (scene_t *)calloc(1, sizeof(scene_t));
  s->ncap = ncap;
  s->nsph = nsph;
  s->nbox = nbox;
  s->cap = (capsule_t *)malloc(sizeof(capsule_t) * (ncap > 0 ? ncap : 1));
  for (int i = 0; i < ncap; ++i) {
    memcpy(s->cap[i].a, caps + 7 * i, 3 * sizeof(double));
    memcpy(s->cap[i].b, caps + 7 * i + 3, 3 * sizeof(double));
    s->cap[i].r = caps[7 * i + 6];
  }
  s->sph = (double *)malloc(sizeof(double) * 4 * (nsph > 0 ? nsph : 1));
  if (nsph) memcpy(s->sph, sph, sizeof(double) * 4 * nsph);
  s->box = (double *)malloc(sizeof(double) * 6 * (nbox > 0 ? nbox : 1));
  if (nbox) memcpy(s->box, box, sizeof(double) * 6 * nbox);
  s->cell = cell;
  s->cell_start = NULL;
  s->cell_items = NULL;
  if (ncap > 0) {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < ncap; ++i)
      for (int k = 0; k < 3; ++k) {
        double a = s->cap[i].a[k], b = s->cap[i].b[k], r = s->cap[i].r;
        double mn = (a < b ? a : b) - r, mx = (a > b ? a : b) + r;
        if (mn < lo[k]) lo[k] = mn;
        if (mx > hi[k]) hi[k] = mx;
      }
    for (int k = 0; k < 3; ++k) {
      s->lo[k] = lo[k] - cell;
      s->dim[k] = (int)ceil((hi[k] + cell - s->lo[k]) / cell);
      if (s->dim[k] < 1) s->dim[k] = 1;
    }
    long ncell = (long)s->dim[0] * s->dim[1] * s->dim[2];
    int *count = (int *)calloc(ncell + 1, sizeof(int));
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        s->cell_start = (int *)calloc(ncell + 1, sizeof(int));
        for (long c = 0; c < ncell; ++c) s->cell_start[c + 1] = s->cell_start[c] + count[c];
        s->cell_items = (int *)malloc(sizeof(int) * (s->cell_start[ncell] + 1));
        memset(count, 0, sizeof(int) * (ncell + 1));
      }
      for (int i = 0; i < ncap; ++i) {
        int c0[3], c1[3];
        for (int k = 0; k < 3; ++k) {
          double a = s->cap[i].a[k], b = s->cap[i].b[k], r = s->cap[i].r;
          double mn = (a < b ? a : b) - r, mx = (a > b ? a : b) + r;
          c0[k] = clampi((int)floor((mn - s->lo[k]) / cell), 0, s->dim[k] - 1);
          c1[k] = clampi((int)floor((mx - s->lo[k]) / cell), 0, s->dim[k] - 1);
        }
        for (int z = c0[2]; z <= c1[2]; ++z)
          for (int y = c0[1]; y <= c1[1]; ++y)
            for (int x = c0[0]; x <= c1[0]; ++x) {
              long c = ((long)z * s->dim[1] + y) * s->dim[0] + x;
              if (pass == 0)
                count[c]++;
              else
                s->cell_items[s->cell_start[c] + count[c]++] = i;
            }
      }
    }
    free(count);
  }
  return s;
}

void rc_destroy(void *h) {
  scene_t *s = (scene_t *)h;
  if (!s) return;
  free(s->cap);
  free(s->sph);
  free(s->box);
  free(s->cell_start);
  free(s->cell_items);
  free(s);
}

/* Walk the capsule grid along the ray (Amanatides-Woo traversal). */
static double hit_capsules_grid(const scene_t *s, const double *o,
                                const double *d, double tmax) {
  double best = INFINITY;
  /* clip the ray to the grid box */
  double gb[6];
  for (int k = 0; k < 3; ++k) {
    gb[k] = s->lo[k];
    gb[3 + k] = s->lo[k] + s->cell * s->dim[k];
  }
  double t0 = 0.0, t1 = tmax;
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0.0) {
      if (o[k] < gb[k] || o[k] > gb[3 + k]) return INFINITY;
      continue;
    }
    double inv = 1.0 / d[k];
    double ta = (gb[k] - o[k]) * inv, tb = (gb[3 + k] - o[k]) * inv;
    if (ta > tb) {
      double t = ta;
      ta = tb;
      tb = t;
    }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
  }
  if (t0 > t1) return INFINITY;
  double p[3];
  int c[3], step[3];
  double tnext[3], tdelta[3];
  for (int k = 0; k < 3; ++k) {
    p[k] = o[k] + d[k] * t0;
    c[k] = clampi((int)floor((p[k] - s->lo[k]) / s->cell), 0, s->dim[k] - 1);
    if (d[k] > 0) {
      step[k] = 1;
      tnext[k] = t0 + ((s->lo[k] + (c[k] + 1) * s->cell) - p[k]) / d[k];
      tdelta[k] = s->cell / d[k];
    } else if (d[k] < 0) {
      step[k] = -1;
      tnext[k] = t0 + ((s->lo[k] + c[k] * s->cell) - p[k]) / d[k];
      tdelta[k] = -s->cell / d[k];
    } else {
      step[k] = 0;
      tnext[k] = INFINITY;
      tdelta[k] = INFINITY;
    }
  }
  for (;;) {
    long ci = ((long)c[2] * s->dim[1] + c[1]) * s->dim[0] + c[0];
    for (int j = s->cell_start[ci]; j < s->cell_start[ci + 1]; ++j) {
      double t = hit_capsule(o, d, &s->cap[s->cell_items[j]], 1e-9);
      if (t < best) best = t;
    }
    int k = 0;
    if (tnext[1] < tnext[k]) k = 1;
    if (tnext[2] < tnext[k]) k = 2;
    if (best <= tnext[k]) break; /* nothing later can be nearer */
    if (tnext[k] > t1) break;
    c[k] += step[k];
    if (c[k] < 0 || c[k] >= s->dim[k]) break;
    tnext[k] += tdelta[k];
  }
  return best;
}

static double cast(const scene_t *s, const double *o, const double *d,
                   double tmax) {
  double best = INFINITY;
  for (int i = 0; i < s->nsph; ++i) {
    double t = hit_sphere(o, d, s->sph + 4 * i, s->sph[4 * i + 3], 1e-9);
    if (t < best) best = t;
  }
  for (int i = 0; i < s->nbox; ++i) {
    double t = hit_box(o, d, s->box + 6 * i, 1e-9);
    if (t < best) best = t;
  }
  if (s->ncap > 0) {
    double t = hit_capsules_grid(s, o, d, tmax);
    if (t < best) best = t;
  }
  return best <= tmax ? best : INFINITY;
}

/* Radical inverse of index i in the given base (Halton sequence). */
static double halton(uint64_t i, uint64_t base) {
  double f = 1.0, r = 0.0;
  while (i > 0) {
    f /= (double)base;
    r += f * (double)(i % base);
    i /= base;
  }
  return r;
}

static inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/* Standard normal from a counter (Box-Muller on two 53-bit uniforms). */
static double gauss(uint64_t seed, uint64_t frame, uint64_t ray) {
  uint64_t k = splitmix64(seed ^ splitmix64(frame * 0xD1B54A32D192ED03ull ^
                                            splitmix64(ray)));
  uint64_t k2 = splitmix64(k);
  double u1 = ((double)(k >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  double u2 = (double)(k2 >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/*
 * Cast Halton-pattern rays from `origin` until `n_hits` hits are collected or
 * `max_rays` rays were cast.  Ray g (global index ray0 + i) points at azimuth
 * 2*pi*H2(g) and elevation el_lo + (el_hi - el_lo)*H3(g).  Writes hit points
 * (float32 xyz) to out, the number of rays consumed to *rays_used; returns the
 * number of hits written.
 */
long rc_frame(void *h, const double *origin, double el_lo, double el_hi,
              uint64_t ray0, long n_hits, double sigma, uint64_t seed,
              uint64_t frame, double max_range, long max_rays, float *out,
              uint64_t *rays_used) {
  const scene_t *s = (const scene_t *)h;
  const long batch = 16384;
  double *tb = (double *)malloc(sizeof(double) * batch);
  long got = 0, cast_n = 0;
  while (got < n_hits && cast_n < max_rays) {
    long nb = batch;
    if (cast_n + nb > max_rays) nb = max_rays - cast_n;
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < nb; ++i) {
      uint64_t g = ray0 + (uint64_t)(cast_n + i);
      double az = 6.283185307179586 * halton(g + 1, 2);
      double el = el_lo + (el_hi - el_lo) * halton(g + 1, 3);
      double d[3] = {cos(el) * cos(az), cos(el) * sin(az), sin(el)};
      tb[i] = cast(s, origin, d, max_range);
    }
    long i = 0;
    for (; i < nb && got < n_hits; ++i) {
      if (!isfinite(tb[i])) continue;
      uint64_t g = ray0 + (uint64_t)(cast_n + i);
      double az = 6.283185307179586 * halton(g + 1, 2);
      double el = el_lo + (el_hi - el_lo) * halton(g + 1, 3);
      double d[3] = {cos(el) * cos(az), cos(el) * sin(az), sin(el)};
      double t = tb[i];
      if (sigma > 0) t += sigma * gauss(seed, frame, g);
      if (t < 1e-3) t = 1e-3;
      for (int k = 0; k < 3; ++k) out[3 * got + k] = (float)(origin[k] + t * d[k]);
      got++;
    }
    cast_n += i;
  }
  free(tb);
  *rays_used = (uint64_t)cast_n;
  return got;
}

/* Noise-free first-hit distances for given unit directions (test helper). */
void rc_cast_many(void *h, const double *origin, const double *dirs, long n,
                  double max_range, double *t_out) {
  const scene_t *s = (const scene_t *)h;
#pragma omp parallel for schedule(dynamic, 256)
  for (long i = 0; i < n; ++i) t_out[i] = cast(s, origin, dirs + 3 * i, max_range);
}
