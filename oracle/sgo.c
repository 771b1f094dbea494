/*
 * sgo.c -- FP64 CPU oracle for bricked, multiresolution, emission-absorption
 * direct volume ray casting (syGlass, arXiv 1804.08197, Section 5).
 *
 * TEST INFRASTRUCTURE. This file is the slow, obviously correct reference the
 * GPU library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no source with the GPU
 * library: no headers, helpers, tables or constants.
 *
 * Every quantity is IEEE double. Build with -O2 -ffp-contract=off and without
 * -ffast-math so that every operation below is rounded exactly as written
 * (the LOD criterion must be reproducible bit for bit).
 *
 * Steps (each function cites the passage it follows):
 *   O2 pyramid            Sec 5.2 (blocks stored in a multi-resolution pyramid)
 *   O3 bricks / min-max   Sec 5.2, Sec 4.1 (blocks at several resolutions)
 *   O4 transfer function  Sec 5.1 (tau[f] emission, T[f] opacity), Sec 8
 *   O5 trilinear sample   Sec 5.1 (3D textures with trilinear filtering)
 *   O6 rays               Sec 5.1 (one ray per pixel), Sec 5.3 (per eye)
 *   O7 entry / exit       Sec 5.1 (x0, x1 of the two integrals)
 *   O8 LOD cut            Sec 5.2 (top-down traversal, angular resolution test)
 *   O9 empty nodes        all-zero opacity over a node's value range
 *   O10 segments          Sec 5.2 (blocks rendered front to back, ray continued)
 *   O11 integration       Sec 5.1 emission-absorption integral, early termination
 *   O12 channels          Sec 8 (multi-channel intensity)
 *   O13 output            Sec 5.6 (alpha channel, pre-multiplied colour)
 *   O15 wrapped-space rays Sec 5.3 (rays spread uniformly over the wrapped image)
 *   O16 ray clipping      Sec 6 (cut plane tool, ROI tool), Sec 5.6 (rays
 *                         ending at the depth of opaque geometry)
 *   O18 residency fallback Sec 5.2 (children missing from the cache are
 *                         requested and the parent is rendered), Sec 4.2
 *                         (least-recently-used chunk cache)
 *   O17 optical models    Sec 5.1 (emission-only, maximum intensity
 *                         projection, emission-absorption), Sec 5.6 (zero
 *                         alpha of the emission-only image)
 *
 * Parity status: every function here is pinned by a CPU test (closed forms,
 * library special cases, brute force); the full-image renders of the
 * synthetic workloads have no printed values in the paper to compare with
 * ("parity unpinned" for whole images beyond the pinned properties).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SGO_MAX_LEVELS 16
#define SGO_MAX_CHANNELS 4

/* ------------------------------------------------------------------ types */

typedef struct {
  double cam_to_world[16]; /* row-major 4x4; eye = (m[3], m[7], m[11]) */
  double tan_left, tan_right, tan_bottom, tan_top;
  int32_t width, height;
  double lens[4]; /* k1, k2, cx, cy of the wrapped-space ray map (O15);
                     k1 = k2 = 0: rectilinear */
} sgo_view;

typedef struct {
  int32_t dims[3];  /* level-0 voxels, x fastest */
  int32_t brick;    /* core edge B of a brick, in voxels of its level */
  int32_t levels;   /* number of pyramid levels */
  int32_t channels;
  int32_t bpv;      /* bytes per voxel: 1 (u8) or 2 (u16) */
  int32_t tf_n;     /* entries per transfer function table */
  const void *const *lvl; /* [channel * levels + L] level arrays, x fastest */
  const double *tf;       /* [channel][tf_n][4]: r, g, b, extinction */
  const double *tf_lo;    /* [channel] raw value mapped to entry 0 */
  const double *tf_hi;    /* [channel] raw value mapped to entry tf_n-1 */
} sgo_scene;

typedef struct {
  double step;        /* step in voxels of the sampled level (0.5) */
  double ert;         /* early termination when accumulated alpha >= ert */
  double tau;         /* LOD: tolerated screen-space voxel size in pixels */
  double bg[4];       /* premultiplied background RGBA */
  double depth_alpha; /* depth output: first sample with alpha >= this */
  int32_t bias;       /* finest level used (0 = full resolution) */
  int32_t lod_on;     /* 1: screen-space LOD cut; 0: every node at level bias */
  int32_t skip_empty; /* 1: drop segments of empty nodes */
  int32_t pad;
  int32_t model;      /* O17: 0 emission-absorption, 1 emission-only,
                         2 maximum intensity projection */
  int32_t n_planes;   /* O16: cut planes in use, 0..4 */
  double planes[4][4]; /* plane j keeps the points p with
                          (n . p) + w <= 0, stored (nx, ny, nz, w) */
  int32_t roi_on;     /* O16: 1 = keep only the box roi */
  int32_t pad2;
  double roi[6];      /* lo x, y, z, hi x, y, z (level-0 units) */
} sgo_params;

/* ------------------------------------------------------------ small utils */

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

static double voxel(const void *a, int bpv, const int64_t n[3], int64_t i,
                    int64_t j, int64_t k) {
  int64_t idx = (k * n[1] + j) * n[0] + i;
  if (bpv == 1) return (double)((const uint8_t *)a)[idx];
  return (double)((const uint16_t *)a)[idx];
}

/* Level dimensions: n_L = ceil(n_{L-1} / 2). */
void sgo_level_dims(const int32_t dims0[3], int32_t L, int32_t out[3]) {
  for (int a = 0; a < 3; ++a) {
    int64_t n = dims0[a];
    for (int l = 0; l < L; ++l) n = (n + 1) / 2;
    out[a] = (int32_t)n;
  }
}

/* Number of bricks per axis at level L: ceil(n_L / B). */
void sgo_brick_grid(const int32_t dims0[3], int32_t B, int32_t L,
                    int32_t out[3]) {
  int32_t n[3];
  sgo_level_dims(dims0, L, n);
  for (int a = 0; a < 3; ++a) out[a] = (n[a] + B - 1) / B;
}

/* Node identifier: level in bits 60..63, brick x in 40..59, y in 20..39,
 * z in 0..19. Sorting identifiers gives a canonical order for comparison. */
uint64_t sgo_node_id(int32_t L, int32_t bx, int32_t by, int32_t bz) {
  return ((uint64_t)L << 60) | ((uint64_t)bx << 40) | ((uint64_t)by << 20) |
         (uint64_t)bz;
}

void sgo_node_decode(uint64_t id, int32_t out[4]) {
  out[0] = (int32_t)(id >> 60);
  out[1] = (int32_t)((id >> 40) & 0xFFFFF);
  out[2] = (int32_t)((id >> 20) & 0xFFFFF);
  out[3] = (int32_t)(id & 0xFFFFF);
}

/* Axis-aligned box of node (L, b) in level-0 units, clipped to the volume:
 * [B 2^L b, B 2^L (b+1)] intersected with [0, dims]. */
void sgo_node_box(const int32_t dims0[3], int32_t B, int32_t L,
                  const int32_t b[3], double lo[3], double hi[3]) {
  for (int a = 0; a < 3; ++a) {
    int64_t w = (int64_t)B << L;
    int64_t l = w * b[a];
    int64_t h = w * (b[a] + 1);
    if (h > dims0[a]) h = dims0[a];
    lo[a] = (double)l;
    hi[a] = (double)h;
  }
}

/* O18 (Sec 5.2: blocks no ray can see are left out): does box [lo, hi]
 * lie outside every ray of the view? The rays leave the eye inside the
 * pyramid spanned by the image's edge tangents (every pixel centre lies
 * half a pixel inside it), so a box whose eight corners all lie beyond one
 * of the four side planes meets none of them. In the camera frame (x
 * right, y up, looking down -z) a corner q lies beyond the right plane when
 * x > tan_right z, with z = -q.z the distance along the view axis. A view
 * with a lens map is never culled: its rays leave the pyramid. */
int32_t sgo_box_outside_view(const sgo_view *v, const double lo[3],
                             const double hi[3]) {
  if (v->lens[0] != 0.0 || v->lens[1] != 0.0) return 0;
  const double *m = v->cam_to_world;
  int nr = 0, nl = 0, nt = 0, nb = 0;
  for (int k = 0; k < 8; ++k) {
    double q0 = ((k & 1) ? hi[0] : lo[0]) - m[3];
    double q1 = ((k & 2) ? hi[1] : lo[1]) - m[7];
    double q2 = ((k & 4) ? hi[2] : lo[2]) - m[11];
    double x = (q0 * m[0] + q1 * m[4]) + q2 * m[8];
    double y = (q0 * m[1] + q1 * m[5]) + q2 * m[9];
    double z = -((q0 * m[2] + q1 * m[6]) + q2 * m[10]);
    nr += x > v->tan_right * z;
    nl += x < v->tan_left * z;
    nt += y > v->tan_top * z;
    nb += y < v->tan_bottom * z;
  }
  return nr == 8 || nl == 8 || nt == 8 || nb == 8;
}

/* ------------------------------------------------------------- O2 pyramid */

/* Next pyramid level (Sec 5.2, multi-resolution pyramid): each coarse voxel
 * is the mean of its 2x2x2 children, children indices clamped to the fine
 * level, rounded half up in integers: (sum + 4) >> 3. */
void sgo_downsample(const void *src, int32_t bpv, const int32_t n[3],
                    void *dst) {
  int64_t fn[3] = {n[0], n[1], n[2]};
  int64_t m[3] = {(n[0] + 1) / 2, (n[1] + 1) / 2, (n[2] + 1) / 2};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m[2]; ++k)
    for (int64_t j = 0; j < m[1]; ++j)
      for (int64_t i = 0; i < m[0]; ++i) {
        uint32_t sum = 0;
        for (int dz = 0; dz < 2; ++dz)
          for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
              sum += (uint32_t)voxel(src, bpv, fn,
                                     clampi(2 * i + dx, 0, fn[0] - 1),
                                     clampi(2 * j + dy, 0, fn[1] - 1),
                                     clampi(2 * k + dz, 0, fn[2] - 1));
        uint32_t v = (sum + 4u) >> 3;
        int64_t o = (k * m[1] + j) * m[0] + i;
        if (bpv == 1)
          ((uint8_t *)dst)[o] = (uint8_t)v;
        else
          ((uint16_t *)dst)[o] = (uint16_t)v;
      }
}

/* ------------------------------------------------- O3 bricks and min-max */

/* Stored region of brick b at a level: voxels [B b - 1, B b + B] per axis,
 * indices clamped to the level, i.e. a core of B^3 plus a one-voxel apron
 * replicated at the volume border. out is (B+2)^3, x fastest. */
void sgo_brick_region(const void *lvl, int32_t bpv, const int32_t n[3],
                      int32_t B, const int32_t b[3], void *out) {
  int64_t ln[3] = {n[0], n[1], n[2]};
  int64_t S = B + 2;
  for (int64_t z = 0; z < S; ++z)
    for (int64_t y = 0; y < S; ++y)
      for (int64_t x = 0; x < S; ++x) {
        double v = voxel(lvl, bpv, ln,
                         clampi((int64_t)B * b[0] - 1 + x, 0, ln[0] - 1),
                         clampi((int64_t)B * b[1] - 1 + y, 0, ln[1] - 1),
                         clampi((int64_t)B * b[2] - 1 + z, 0, ln[2] - 1));
        int64_t o = (z * S + y) * S + x;
        if (bpv == 1)
          ((uint8_t *)out)[o] = (uint8_t)v;
        else
          ((uint16_t *)out)[o] = (uint16_t)v;
      }
}

/* Minimum and maximum over the stored (B+2)^3 region of brick b. */
void sgo_brick_minmax(const void *lvl, int32_t bpv, const int32_t n[3],
                      int32_t B, const int32_t b[3], double *mn, double *mx) {
  int64_t ln[3] = {n[0], n[1], n[2]};
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t z = -1; z <= B; ++z)
    for (int64_t y = -1; y <= B; ++y)
      for (int64_t x = -1; x <= B; ++x) {
        double v = voxel(lvl, bpv, ln,
                         clampi((int64_t)B * b[0] + x, 0, ln[0] - 1),
                         clampi((int64_t)B * b[1] + y, 0, ln[1] - 1),
                         clampi((int64_t)B * b[2] + z, 0, ln[2] - 1));
        if (v < lo) lo = v;
        if (v > hi) hi = v;
      }
  *mn = lo;
  *mx = hi;
}

/* ------------------------------------------------- O4 transfer function */

/* Continuous table index of raw value v: (v - lo)/(hi - lo) * (N - 1),
 * before clamping. Entry k sits at k/(N-1) of the domain [lo, hi]. */
static double tf_index(double v, double lo, double hi, int32_t N) {
  return ((v - lo) / (hi - lo)) * (double)(N - 1);
}

/* Transfer function (Sec 5.1: c = tau[f], rho = T[f]; Sec 8: linear maps,
 * palettes): linear interpolation between table entries, clamped at both
 * ends. Channels 0..2 are the emitted colour tau, channel 3 the extinction
 * rho per level-0 voxel length. */
void sgo_tf_eval(const double *tf, int32_t N, double lo, double hi, double v,
                 double out[4]) {
  double u = tf_index(v, lo, hi, N);
  if (u < 0.0) u = 0.0;
  if (u > (double)(N - 1)) u = (double)(N - 1);
  int32_t k0 = (int32_t)floor(u);
  int32_t k1 = k0 + 1 < N ? k0 + 1 : N - 1;
  double w = u - (double)k0;
  for (int c = 0; c < 4; ++c)
    out[c] = (1.0 - w) * tf[4 * k0 + c] + w * tf[4 * k1 + c];
}

/* ---------------------------------------------------- O5 trilinear sample */

/* Trilinear reconstruction at world point p (level-0 units) from level L
 * (Sec 5.1, 3D textures with trilinear interpolation). Voxel i of level L
 * covers [2^L i, 2^L (i+1)) with its value at the centre; outside the last
 * centres the edge value is held (clamp to edge). */
double sgo_sample(const void *lvl, int32_t bpv, const int32_t n[3], int32_t L,
                  const double p[3]) {
  int64_t ln[3] = {n[0], n[1], n[2]};
  double s = ldexp(1.0, L);
  int64_t i0[3], i1[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double q = p[a] / s - 0.5;
    double fl = floor(q);
    f[a] = q - fl;
    i0[a] = clampi((int64_t)fl, 0, ln[a] - 1);
    i1[a] = clampi((int64_t)fl + 1, 0, ln[a] - 1);
  }
  double c[2][2];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      int64_t y = dy ? i1[1] : i0[1], z = dz ? i1[2] : i0[2];
      double a = voxel(lvl, bpv, ln, i0[0], y, z);
      double b = voxel(lvl, bpv, ln, i1[0], y, z);
      c[dz][dy] = (1.0 - f[0]) * a + f[0] * b;
    }
  double c0 = (1.0 - f[1]) * c[0][0] + f[1] * c[0][1];
  double c1 = (1.0 - f[1]) * c[1][0] + f[1] * c[1][1];
  return (1.0 - f[2]) * c0 + f[2] * c1;
}

/* ------------------------------------------------------------------ O6 */

/* Eye and unit direction of the ray through the centre of pixel (x, y),
 * y = 0 the top row (Sec 5.1, one ray per pixel). Camera looks down -z of
 * its own frame; cam_to_world maps camera to world (level-0 voxels). */
void sgo_ray(const sgo_view *v, int32_t x, int32_t y, double e[3],
             double d[3]) {
  const double *m = v->cam_to_world;
  double sx = v->tan_left +
              (((double)x + 0.5) / (double)v->width) *
                  (v->tan_right - v->tan_left);
  double sy = v->tan_top -
              (((double)y + 0.5) / (double)v->height) *
                  (v->tan_top - v->tan_bottom);
  /* O15, wrapped space (Sec 5.3): the pixels of the wrapped image are
   * spread uniformly and each is moved, radially about the lens centre
   * (cx, cy), to the tangent the lens shows it at: with r^2 the squared
   * distance from the centre, the offset grows by 1 + k1 r^2 + k2 r^4. */
  if (v->lens[0] != 0.0 || v->lens[1] != 0.0) {
    double dx = sx - v->lens[2], dy = sy - v->lens[3];
    double r2 = dx * dx + dy * dy;
    double f = 1.0 + r2 * (v->lens[0] + r2 * v->lens[1]);
    sx = v->lens[2] + dx * f;
    sy = v->lens[3] + dy * f;
  }
  double w[3];
  for (int a = 0; a < 3; ++a) {
    e[a] = m[4 * a + 3];
    w[a] = (m[4 * a + 0] * sx + m[4 * a + 1] * sy) + m[4 * a + 2] * (-1.0);
  }
  double len = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
  for (int a = 0; a < 3; ++a) d[a] = w[a] / len;
}

/* ------------------------------------------------------------------ O7 */

/* Slab test of the ray e + t d against box [lo, hi]. Writes the parameter
 * interval (not clipped to t >= 0) and returns 1 if it is non-empty.
 * An axis with d = 0 leaves the interval unbounded if the eye lies within
 * the slab and empties it otherwise. */
int32_t sgo_box_interval(const double e[3], const double d[3],
                         const double lo[3], const double hi[3], double *t0,
                         double *t1) {
  double a = -INFINITY, b = INFINITY;
  for (int i = 0; i < 3; ++i) {
    if (d[i] != 0.0) {
      double ta = (lo[i] - e[i]) / d[i];
      double tb = (hi[i] - e[i]) / d[i];
      double mn = ta < tb ? ta : tb;
      double mx = ta < tb ? tb : ta;
      if (mn > a) a = mn;
      if (mx < b) b = mx;
    } else if (!(lo[i] <= e[i] && e[i] <= hi[i])) {
      *t0 = 0.0;
      *t1 = 0.0;
      return 0;
    }
  }
  *t0 = a;
  *t1 = b;
  return a < b;
}

/* Entry x0 and exit x1 of the integrals in Sec 5.1: the ray against the
 * volume box [0, dims], starting at the eye (t >= 0, no near plane). */
int32_t sgo_entry_exit(const int32_t dims0[3], const double e[3],
                       const double d[3], double *tn, double *tf) {
  double lo[3] = {0.0, 0.0, 0.0};
  double hi[3] = {(double)dims0[0], (double)dims0[1], (double)dims0[2]};
  double a, b;
  sgo_box_interval(e, d, lo, hi, &a, &b);
  if (a < 0.0) a = 0.0;
  *tn = a;
  *tf = b;
  return a < b;
}

/* O16 clipping: narrow the ray interval [*t0, *t1] to the part that is
 * kept by every cut plane (Sec 6: the volume is seen as if the portion above
 * the plane were missing), inside the region of interest (Sec 6: data
 * outside the ROI cut out of the rendering) and in front of the opaque
 * geometry at distance `limit` along the ray (Sec 5.6: the ray is
 * terminated at the distance read from the depth texture; +inf = none).
 * Plane j keeps e + t d where a + t b <= 0 with a = (n . e) + w and
 * b = n . d: t <= -a/b for b > 0, t >= -a/b for b < 0, every t or none for
 * b = 0. Returns 1 if the interval stays non-empty. */
int32_t sgo_clip(const sgo_params *pr, const double e[3], const double d[3],
                 double limit, double *t0, double *t1) {
  double a0 = *t0, a1 = *t1;
  for (int32_t j = 0; j < pr->n_planes; ++j) {
    const double *q = pr->planes[j];
    double a = ((q[0] * e[0] + q[1] * e[1]) + q[2] * e[2]) + q[3];
    double b = (q[0] * d[0] + q[1] * d[1]) + q[2] * d[2];
    if (b > 0.0) {
      double t = -a / b;
      if (t < a1) a1 = t;
    } else if (b < 0.0) {
      double t = -a / b;
      if (t > a0) a0 = t;
    } else if (a > 0.0) {
      a1 = a0;
    }
  }
  if (pr->roi_on) {
    double r0, r1;
    if (!sgo_box_interval(e, d, pr->roi, pr->roi + 3, &r0, &r1)) {
      a1 = a0;
    } else {
      if (r0 > a0) a0 = r0;
      if (r1 < a1) a1 = r1;
    }
  }
  if (limit < a1) a1 = limit;
  *t0 = a0;
  *t1 = a1;
  return a0 < a1;
}

/* ------------------------------------------------------------------ O8 */

/* Pixel angle and LOD constant: theta = (tan_top - tan_bottom) / H and
 * K = (tau theta)^2. */
double sgo_lod_k(const sgo_view *v, double tau) {
  double theta = (v->tan_top - v->tan_bottom) / (double)v->height;
  return (tau * theta) * (tau * theta);
}

/* LOD acceptance of node (L, b) for eye e (Sec 5.2: a block suits when the
 * angular size of its voxels at the distance of its closest face does not
 * exceed the angular size of a pixel). With d the distance from the eye to
 * the nearest point of the node box and s = 2^L the voxel edge:
 *   accept  <=>  L == bias  or  s*s <= K * d*d.
 * Operations in exactly this order. */
int32_t sgo_node_accept(const int32_t dims0[3], int32_t B, const double e[3],
                        double K, int32_t bias, int32_t L,
                        const int32_t b[3]) {
  if (L == bias) return 1;
  double lo[3], hi[3];
  sgo_node_box(dims0, B, L, b, lo, hi);
  double dl[3];
  for (int a = 0; a < 3; ++a) {
    double u = lo[a] - e[a];
    double w = e[a] - hi[a];
    double m = u > w ? u : w;
    dl[a] = m > 0.0 ? m : 0.0;
  }
  double d2 = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
  double s = ldexp(1.0, L);
  return (s * s) <= (K * d2);
}

typedef struct {
  const int32_t *dims0;
  int32_t B, bias, lod_on;
  const double *e;
  double K;
  uint64_t *out;
  int64_t n, cap;
  int32_t grid[SGO_MAX_LEVELS][3];
} cut_ctx;

static void cut_visit(cut_ctx *c, int32_t L, const int32_t b[3]) {
  int32_t acc = c->lod_on ? sgo_node_accept(c->dims0, c->B, c->e, c->K,
                                            c->bias, L, b)
                          : (L == c->bias);
  if (acc) {
    if (c->n < c->cap) c->out[c->n] = sgo_node_id(L, b[0], b[1], b[2]);
    c->n++;
    return;
  }
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int32_t cb[3] = {2 * b[0] + dx, 2 * b[1] + dy, 2 * b[2] + dz};
        if (cb[0] < c->grid[L - 1][0] && cb[1] < c->grid[L - 1][1] &&
            cb[2] < c->grid[L - 1][2])
          cut_visit(c, L - 1, cb);
      }
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* LOD cut of one view (Sec 5.2 traversal): start from every node of the top
 * level; a node that suits is registered, otherwise its existing children are
 * visited. Returns the number of cut nodes (the first cap are written,
 * sorted ascending by identifier); -1 on bad arguments. */
int64_t sgo_lod_cut(const int32_t dims0[3], int32_t B, int32_t levels,
                    const sgo_view *v, double tau, int32_t bias,
                    int32_t lod_on, uint64_t *out, int64_t cap) {
  if (levels < 1 || levels > SGO_MAX_LEVELS || bias < 0 || bias >= levels)
    return -1;
  cut_ctx c;
  c.dims0 = dims0;
  c.B = B;
  c.bias = bias;
  c.lod_on = lod_on;
  double e[3] = {v->cam_to_world[3], v->cam_to_world[7], v->cam_to_world[11]};
  c.e = e;
  c.K = sgo_lod_k(v, tau);
  c.out = out;
  c.n = 0;
  c.cap = cap;
  for (int32_t L = 0; L < levels; ++L) sgo_brick_grid(dims0, B, L, c.grid[L]);
  int32_t T = levels - 1;
  for (int32_t z = 0; z < c.grid[T][2]; ++z)
    for (int32_t y = 0; y < c.grid[T][1]; ++y)
      for (int32_t x = 0; x < c.grid[T][0]; ++x) {
        int32_t b[3] = {x, y, z};
        cut_visit(&c, T, b);
      }
  if (out && c.n <= cap) qsort(out, (size_t)c.n, sizeof(uint64_t), cmp_u64);
  return c.n;
}

/* O18: the cut when only some nodes are in the GPU cache (Sec 5.2). The
 * traversal above with one change: a node that is too coarse for the view
 * descends only if all of its existing children are resident; otherwise the
 * node itself is drawn, one level coarser than wanted, and the children that
 * are absent are recorded as requests for the loader, except those no ray
 * of the view can see (sgo_box_outside_view).
 * `resident` is the ascending list of resident node identifiers; every
 * top-level node must be in it (returns -2 otherwise). The requested
 * identifiers (ascending, without repeats) go to req (first req_cap),
 * their number to *n_req. Returns the cut size as sgo_lod_cut does. */
typedef struct {
  cut_ctx c;
  const sgo_view *v;
  const uint64_t *res;
  int64_t n_res;
  uint64_t *req;
  int64_t n_req, req_cap;
} res_ctx;

static int is_resident(const res_ctx *r, uint64_t id) {
  return bsearch(&id, r->res, (size_t)r->n_res, sizeof(uint64_t), cmp_u64) != NULL;
}

static void res_visit(res_ctx *r, int32_t L, const int32_t b[3]) {
  cut_ctx *c = &r->c;
  int32_t acc = c->lod_on ? sgo_node_accept(c->dims0, c->B, c->e, c->K,
                                            c->bias, L, b)
                          : (L == c->bias);
  int32_t kids[8][3];
  int nk = 0, all_res = 1;
  if (!acc) {
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          int32_t cb[3] = {2 * b[0] + dx, 2 * b[1] + dy, 2 * b[2] + dz};
          if (cb[0] < c->grid[L - 1][0] && cb[1] < c->grid[L - 1][1] &&
              cb[2] < c->grid[L - 1][2]) {
            memcpy(kids[nk++], cb, sizeof(cb));
            if (!is_resident(r, sgo_node_id(L - 1, cb[0], cb[1], cb[2]))) all_res = 0;
          }
        }
  }
  if (acc || !all_res) {
    if (c->n < c->cap) c->out[c->n] = sgo_node_id(L, b[0], b[1], b[2]);
    c->n++;
    for (int k = 0; k < nk; ++k) {
      uint64_t id = sgo_node_id(L - 1, kids[k][0], kids[k][1], kids[k][2]);
      if (is_resident(r, id)) continue;
      double lo[3], hi[3];
      sgo_node_box(c->dims0, c->B, L - 1, kids[k], lo, hi);
      if (sgo_box_outside_view(r->v, lo, hi)) continue;
      if (r->n_req < r->req_cap) r->req[r->n_req] = id;
      r->n_req++;
    }
    return;
  }
  for (int k = 0; k < nk; ++k) res_visit(r, L - 1, kids[k]);
}

int64_t sgo_lod_cut_resident(const int32_t dims0[3], int32_t B, int32_t levels,
                             const sgo_view *v, double tau, int32_t bias,
                             int32_t lod_on, const uint64_t *resident,
                             int64_t n_resident, uint64_t *out, int64_t cap,
                             uint64_t *req, int64_t req_cap, int64_t *n_req) {
  if (levels < 1 || levels > SGO_MAX_LEVELS || bias < 0 || bias >= levels ||
      !resident || !n_req)
    return -1;
  res_ctx r;
  cut_ctx *c = &r.c;
  c->dims0 = dims0;
  c->B = B;
  c->bias = bias;
  c->lod_on = lod_on;
  double e[3] = {v->cam_to_world[3], v->cam_to_world[7], v->cam_to_world[11]};
  c->e = e;
  c->K = sgo_lod_k(v, tau);
  c->out = out;
  c->n = 0;
  c->cap = cap;
  r.v = v;
  r.res = resident;
  r.n_res = n_resident;
  r.req = req;
  r.n_req = 0;
  r.req_cap = req_cap;
  for (int32_t L = 0; L < levels; ++L) sgo_brick_grid(dims0, B, L, c->grid[L]);
  int32_t T = levels - 1;
  for (int32_t z = 0; z < c->grid[T][2]; ++z)
    for (int32_t y = 0; y < c->grid[T][1]; ++y)
      for (int32_t x = 0; x < c->grid[T][0]; ++x)
        if (!is_resident(&r, sgo_node_id(T, x, y, z))) return -2;
  for (int32_t z = 0; z < c->grid[T][2]; ++z)
    for (int32_t y = 0; y < c->grid[T][1]; ++y)
      for (int32_t x = 0; x < c->grid[T][0]; ++x) {
        int32_t b[3] = {x, y, z};
        res_visit(&r, T, b);
      }
  if (out && c->n <= cap) qsort(out, (size_t)c->n, sizeof(uint64_t), cmp_u64);
  /* every node has one parent, so no request appears twice; sorting gives
   * the canonical order */
  if (req && r.n_req <= req_cap) qsort(req, (size_t)r.n_req, sizeof(uint64_t), cmp_u64);
  *n_req = r.n_req;
  return c->n;
}

/* ------------------------------------------------------------------ O9 */

/* A node is empty when, for every channel, the extinction of every table
 * entry that a sample inside it can touch is exactly zero. The value range
 * [min, max] of its stored voxels maps to [u_min, u_max]; entries
 * floor(u_min) - 1 .. floor(u_max) + 2 (clamped) are checked. The extra
 * entry on each side keeps the test valid when the sampler evaluates the
 * table index in a lower precision. Every sample of an empty node then has
 * rho = 0, contributes alpha = 0, and skipping it changes no result. */
int32_t sgo_node_empty(const sgo_scene *sc, int32_t L, const int32_t b[3]) {
  int32_t n[3];
  sgo_level_dims(sc->dims, L, n);
  int32_t N = sc->tf_n;
  for (int32_t ch = 0; ch < sc->channels; ++ch) {
    double mn, mx;
    sgo_brick_minmax(sc->lvl[ch * sc->levels + L], sc->bpv, n, sc->brick, b,
                     &mn, &mx);
    double lo = sc->tf_lo[ch], hi = sc->tf_hi[ch];
    double umin = tf_index(mn, lo, hi, N);
    double umax = tf_index(mx, lo, hi, N);
    int64_t klo = clampi((int64_t)floor(umin) - 1, 0, N - 1);
    int64_t khi = clampi((int64_t)floor(umax) + 2, 0, N - 1);
    const double *t = sc->tf + (size_t)ch * N * 4;
    for (int64_t k = klo; k <= khi; ++k)
      if (t[4 * k + 3] != 0.0) return 0;
  }
  return 1;
}

/* The emission-only counterpart (O17): a node is dark when, for every
 * channel, the emitted colour (r, g, b) of every table entry a sample in it
 * can touch (the same guarded entry range as above) is exactly zero; its
 * samples then add nothing to the emission integral. */
int32_t sgo_node_dark(const sgo_scene *sc, int32_t L, const int32_t b[3]) {
  int32_t n[3];
  sgo_level_dims(sc->dims, L, n);
  int32_t N = sc->tf_n;
  for (int32_t ch = 0; ch < sc->channels; ++ch) {
    double mn, mx;
    sgo_brick_minmax(sc->lvl[ch * sc->levels + L], sc->bpv, n, sc->brick, b,
                     &mn, &mx);
    double lo = sc->tf_lo[ch], hi = sc->tf_hi[ch];
    int64_t klo = clampi((int64_t)floor(tf_index(mn, lo, hi, N)) - 1, 0, N - 1);
    int64_t khi = clampi((int64_t)floor(tf_index(mx, lo, hi, N)) + 2, 0, N - 1);
    const double *t = sc->tf + (size_t)ch * N * 4;
    for (int64_t k = klo; k <= khi; ++k)
      if (t[4 * k] != 0.0 || t[4 * k + 1] != 0.0 || t[4 * k + 2] != 0.0)
        return 0;
  }
  return 1;
}

/* Empty flags for a list of node identifiers: model 0 (emission-absorption)
 * tests the extinction (sgo_node_empty), model 1 (emission-only) the
 * emitted colour (sgo_node_dark); model 2 (maximum intensity) has none. */
void sgo_nodes_empty_model(const sgo_scene *sc, int32_t model,
                           const uint64_t *ids, int64_t n, uint8_t *out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    int32_t q[4];
    sgo_node_decode(ids[i], q);
    int32_t b[3] = {q[1], q[2], q[3]};
    out[i] = model == 0 ? (uint8_t)sgo_node_empty(sc, q[0], b)
             : model == 1 ? (uint8_t)sgo_node_dark(sc, q[0], b)
                          : 0;
  }
}

void sgo_nodes_empty(const sgo_scene *sc, const uint64_t *ids, int64_t n,
                     uint8_t *out) {
  sgo_nodes_empty_model(sc, 0, ids, n, out);
}

/* ---------------------------------------------------------- O10 .. O13 */

typedef struct {
  double t0, t1;
  uint64_t id;
  int64_t idx; /* position in the cut */
  int32_t L;
} seg_t;

static int cmp_seg(const void *a, const void *b) {
  const seg_t *x = (const seg_t *)a, *y = (const seg_t *)b;
  if (x->t0 < y->t0) return -1;
  if (x->t0 > y->t0) return 1;
  return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* Mark the 4^3 micro-blocks of level L touched by the trilinear stencil at
 * p (counter for the memory traffic the method needs). */
static void mark_microblocks(uint8_t *bm, const int32_t n[3], int32_t L,
                             const double p[3]) {
  double s = ldexp(1.0, L);
  int64_t lo[3], hi[3], m[3];
  for (int a = 0; a < 3; ++a) {
    double q = p[a] / s - 0.5;
    int64_t fl = (int64_t)floor(q);
    lo[a] = clampi(fl, 0, n[a] - 1) >> 2;
    hi[a] = clampi(fl + 1, 0, n[a] - 1) >> 2;
    m[a] = (n[a] + 3) / 4;
  }
  for (int64_t z = lo[2]; z <= hi[2]; ++z)
    for (int64_t y = lo[1]; y <= hi[1]; ++y)
      for (int64_t x = lo[0]; x <= hi[0]; ++x) {
#pragma omp atomic write
        bm[(z * m[1] + y) * m[0] + x] = 1;
      }
}

/* Colour and extinction of one sample: per channel transfer function, then
 * additive combination (Sec 8, multi-channel intensity): rho = sum rho_c and
 * rgb = sum(rho_c rgb_c) / rho (zero when rho = 0). */
static void shade(const sgo_scene *sc, int32_t L, const double p[3],
                  double rgb[3], double *rho, uint8_t *const *mb) {
  int32_t n[3];
  sgo_level_dims(sc->dims, L, n);
  if (sc->channels == 1) {
    double v = sgo_sample(sc->lvl[L], sc->bpv, n, L, p);
    double o[4];
    sgo_tf_eval(sc->tf, sc->tf_n, sc->tf_lo[0], sc->tf_hi[0], v, o);
    rgb[0] = o[0];
    rgb[1] = o[1];
    rgb[2] = o[2];
    *rho = o[3];
    if (mb) mark_microblocks(mb[L], n, L, p);
    return;
  }
  double r = 0.0, acc[3] = {0.0, 0.0, 0.0};
  for (int32_t ch = 0; ch < sc->channels; ++ch) {
    double v = sgo_sample(sc->lvl[ch * sc->levels + L], sc->bpv, n, L, p);
    double o[4];
    sgo_tf_eval(sc->tf + (size_t)ch * sc->tf_n * 4, sc->tf_n, sc->tf_lo[ch],
                sc->tf_hi[ch], v, o);
    r += o[3];
    for (int c = 0; c < 3; ++c) acc[c] += o[3] * o[c];
    if (mb) mark_microblocks(mb[ch * sc->levels + L], n, L, p);
  }
  *rho = r;
  for (int c = 0; c < 3; ++c) rgb[c] = r > 0.0 ? acc[c] / r : 0.0;
}

/* Per-channel trilinear values of one sample (O5), marking micro-blocks. */
static void sample_channels(const sgo_scene *sc, int32_t L, const double p[3],
                            double v[SGO_MAX_CHANNELS], uint8_t *const *mb) {
  int32_t n[3];
  sgo_level_dims(sc->dims, L, n);
  for (int32_t ch = 0; ch < sc->channels; ++ch) {
    v[ch] = sgo_sample(sc->lvl[ch * sc->levels + L], sc->bpv, n, L, p);
    if (mb) mark_microblocks(mb[ch * sc->levels + L], n, L, p);
  }
}

/* Emitted colour of channel values v: the sum over channels of tau_c(v_c)
 * (Sec 5.1 emission c = tau[f]; Sec 8, channel intensities add). */
static void emission(const sgo_scene *sc, const double v[SGO_MAX_CHANNELS],
                     double rgb[3]) {
  rgb[0] = rgb[1] = rgb[2] = 0.0;
  for (int32_t ch = 0; ch < sc->channels; ++ch) {
    double o[4];
    sgo_tf_eval(sc->tf + (size_t)ch * sc->tf_n * 4, sc->tf_n, sc->tf_lo[ch],
                sc->tf_hi[ch], v[ch], o);
    for (int c = 0; c < 3; ++c) rgb[c] += o[c];
  }
}

/* Render the given pixels of one view.
 *   cut, cut_empty : the view's LOD cut (sgo_lod_cut) and the flags of the
 *                    params' model (sgo_nodes_empty_model)
 *   pix            : npix (x, y) pairs, or NULL for every pixel row-major
 *   limit          : NULL, or the view's width*height ray limits (O16),
 *                    row-major, +inf where there is no geometry
 *   rgba           : npix * 4 premultiplied colour and alpha (O13)
 *   depth          : npix, t of the first sample with alpha >= depth_alpha,
 *                    +inf if none (optional)
 *   nsamp          : npix sample counts (optional)
 *   mb             : [channel * levels + L] micro-block bitmaps (optional)
 * Returns the total number of samples, or -1 on bad arguments.
 *
 * Segments are the cut nodes crossed by the ray inside its clipped interval
 * (O7, O16), in order of entry (front to back, Sec 5.2). Along a segment of
 * level L the step is D = step 2^L level-0 units, n = ceil(len / D) samples
 * at the midpoints of the sub-intervals (the last one partial, length s_k).
 * Per sample (O17):
 *   emission-absorption (Sec 5.1): a = 1 - exp(-rho s_k); C += (1 - A) a rgb;
 *     A += (1 - A) a; the ray stops once A >= ert (early termination);
 *   emission-only (Sec 5.1): C += rgb s_k with rgb the summed emission;
 *     A stays 0 (Sec 5.6), no termination;
 *   maximum intensity: m_c = max(m_c, v_c) per channel; at the end C is the
 *     summed emission of the maxima, A = 0; with skip_empty a node whose
 *     stored maximum cannot raise any m_c is passed over (exact: trilinear
 *     values never exceed the stencil's largest voxel). */
int64_t sgo_render(const sgo_scene *sc, const sgo_view *v, const sgo_params *pr,
                   const uint64_t *cut, int64_t ncut, const uint8_t *cut_empty,
                   int64_t npix, const int32_t *pix, const double *limit,
                   double *rgba, double *depth, int64_t *nsamp,
                   uint8_t *const *mb, int32_t nthreads) {
  if (!sc || !v || !pr || !rgba || sc->channels < 1 ||
      sc->channels > SGO_MAX_CHANNELS || v->width < 1 || v->height < 1 ||
      pr->model < 0 || pr->model > 2 || pr->n_planes < 0 || pr->n_planes > 4)
    return -1;
  int64_t total = (int64_t)v->width * v->height;
  if (!pix) npix = total;
  int64_t sum = 0;
  const int32_t model = pr->model, nch = sc->channels;
  /* stored maxima of the cut nodes, per channel (maximum intensity skip) */
  double *nmax = NULL;
  if (model == 2 && pr->skip_empty && ncut > 0) {
    nmax = (double *)malloc(sizeof(double) * (size_t)(ncut * nch));
    for (int64_t i = 0; i < ncut; ++i) {
      int32_t q[4], n[3];
      sgo_node_decode(cut[i], q);
      int32_t b[3] = {q[1], q[2], q[3]};
      sgo_level_dims(sc->dims, q[0], n);
      for (int32_t ch = 0; ch < nch; ++ch) {
        double mn, mx;
        sgo_brick_minmax(sc->lvl[ch * sc->levels + q[0]], sc->bpv, n, sc->brick,
                         b, &mn, &mx);
        nmax[i * nch + ch] = mx;
      }
    }
  }
  /* the thread count of this call only (the process-wide default stays) */
#ifdef _OPENMP
  const int team = nthreads > 0 ? (int)nthreads : omp_get_max_threads();
#else
  const int team = 1;
  (void)nthreads;
#endif
#pragma omp parallel num_threads(team) reduction(+ : sum)
  {
    seg_t *segs = (seg_t *)malloc(sizeof(seg_t) * (size_t)(ncut > 0 ? ncut : 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
      int32_t x = pix ? pix[2 * p] : (int32_t)(p % v->width);
      int32_t y = pix ? pix[2 * p + 1] : (int32_t)(p / v->width);
      double e[3], d[3], tn, tf;
      sgo_ray(v, x, y, e, d);
      double C[3] = {0.0, 0.0, 0.0}, A = 0.0, dep = INFINITY;
      double vmax[SGO_MAX_CHANNELS];
      int sampled = 0;
      for (int32_t ch = 0; ch < nch; ++ch) vmax[ch] = -INFINITY;
      int64_t ns = 0;
      double lim = limit ? limit[(int64_t)y * v->width + x] : INFINITY;
      if (sgo_entry_exit(sc->dims, e, d, &tn, &tf) &&
          sgo_clip(pr, e, d, lim, &tn, &tf)) {
        int64_t m = 0;
        for (int64_t i = 0; i < ncut; ++i) {
          if (pr->skip_empty && model != 2 && cut_empty && cut_empty[i]) continue;
          int32_t q[4];
          sgo_node_decode(cut[i], q);
          int32_t b[3] = {q[1], q[2], q[3]};
          double lo[3], hi[3], a0, a1;
          sgo_node_box(sc->dims, sc->brick, q[0], b, lo, hi);
          if (!sgo_box_interval(e, d, lo, hi, &a0, &a1)) continue;
          /* a ray that runs inside a face shared by two nodes belongs to
           * the node on the face's upper side (voxel cells are half-open,
           * O1); the volume's own upper faces stay closed */
          int on_face = 0;
          for (int a = 0; a < 3; ++a)
            if (d[a] == 0.0 && e[a] == hi[a] && hi[a] < (double)sc->dims[a]) on_face = 1;
          if (on_face) continue;
          if (a0 < tn) a0 = tn;
          if (a1 > tf) a1 = tf;
          if (!(a0 < a1)) continue;
          segs[m].t0 = a0;
          segs[m].t1 = a1;
          segs[m].id = cut[i];
          segs[m].L = q[0];
          segs[m].idx = i;
          ++m;
        }
        qsort(segs, (size_t)m, sizeof(seg_t), cmp_seg);
        int done = 0;
        for (int64_t i = 0; i < m && !done; ++i) {
          if (nmax && sampled) {
            int raise = 0;
            for (int32_t ch = 0; ch < nch; ++ch)
              if (nmax[segs[i].idx * nch + ch] > vmax[ch]) raise = 1;
            if (!raise) continue;
          }
          int32_t L = segs[i].L;
          double D = pr->step * ldexp(1.0, L);
          double len = segs[i].t1 - segs[i].t0;
          int64_t n = (int64_t)ceil(len / D);
          for (int64_t k = 0; k < n; ++k) {
            double s = D < len - (double)k * D ? D : len - (double)k * D;
            double t = segs[i].t0 + (double)k * D + s / 2.0;
            double pt[3] = {e[0] + t * d[0], e[1] + t * d[1], e[2] + t * d[2]};
            ++ns;
            if (model == 0) {
              double rgb[3], rho;
              shade(sc, L, pt, rgb, &rho, mb);
              double a = 1.0 - exp(-rho * s);
              double w = (1.0 - A) * a;
              for (int c = 0; c < 3; ++c) C[c] += w * rgb[c];
              A += w;
              if (depth && dep == INFINITY && A >= pr->depth_alpha) dep = t;
              if (A >= pr->ert) {
                done = 1;
                break;
              }
            } else {
              double val[SGO_MAX_CHANNELS];
              sample_channels(sc, L, pt, val, mb);
              if (model == 1) {
                double rgb[3];
                emission(sc, val, rgb);
                for (int c = 0; c < 3; ++c) C[c] += rgb[c] * s;
              } else {
                for (int32_t ch = 0; ch < nch; ++ch)
                  if (val[ch] > vmax[ch]) vmax[ch] = val[ch];
                sampled = 1;
              }
            }
          }
        }
      }
      if (model == 2 && sampled) emission(sc, vmax, C);
      double *o = rgba + 4 * p;
      for (int c = 0; c < 3; ++c) o[c] = C[c] + (1.0 - A) * pr->bg[c];
      o[3] = A + (1.0 - A) * pr->bg[3];
      if (depth) depth[p] = dep;
      if (nsamp) nsamp[p] = ns;
      sum += ns;
    }
    free(segs);
  }
  free(nmax);
  return sum;
}

/* Number of threads the OpenMP runtime will use. */
int32_t sgo_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
