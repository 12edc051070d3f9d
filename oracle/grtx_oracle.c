/*
 * grtx_oracle.c -- FP64 brute-force reference for 3D Gaussian ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU path is checked
 * against. It is called by the tests, by the smoke check and by the benchmark's CPU
 * baseline, and by nothing else; the product path never links or calls it. It shares
 * no code, header, table or constant with the GPU library.
 *
 * What it computes is the plain definition of the rendered image, written out without
 * any acceleration structure, blocking or reordering:
 *
 *   - Gaussians (Sec. II-B): mean mu, covariance Sigma = R S S^T R^T with R the
 *     rotation of the normalised quaternion (w,x,y,z) and S = diag(s), opacity o,
 *     real spherical-harmonic colour coefficients.
 *   - Each Gaussian is bounded by the ellipsoid of Mahalanobis radius rho with
 *     rho^2 = 2 ln(o / alpha_min): on that surface o*G = alpha_min ("an ellipsoid with
 *     defined boundaries", Sec. II-B). Gaussians with o <= alpha_min are never hit.
 *   - Every ray is tested against every Gaussian. A hit is a ray that meets the
 *     ellipsoid with entry distance t0 > t_near (the smaller root of the quadric).
 *     Hits are sorted by distance (Sec. III-A: the intersection distance is the depth
 *     used by the k-buffer), ties by Gaussian index.
 *   - Alpha of a hit at the point of maximum response along the ray (Eq. 2):
 *     t_alpha = (mu - o)^T Sigma^-1 d / (d^T Sigma^-1 d), alpha = o * G(o + t_alpha d).
 *   - Colour from SH evaluated at the normalised ray direction (Sec. III-A), offset by
 *     0.5 and clamped at zero.
 *   - Front-to-back compositing (Eq. 1) with early ray termination (Sec. III-A): the
 *     hit that drops transmittance below T_min is still blended, then the ray stops.
 *   - Output: colour C + T*bg, depth sum(w_i t_alpha_i), opacity 1 - T.
 *   - A ray may be bounded by a surface at distance t_far (hits need key < t_far; the
 *     surface hides the background) and may start with a transmittance below one, the
 *     part of the light left after what an earlier ray segment blended.
 *
 * Proxy-key mode orders the same hits by the distance at which the ray enters the
 * Gaussian's bounding icosahedron (20 triangles, inradius 1 in the space where the
 * bounding ellipsoid is the unit sphere), the bounding mesh of the triangle-based
 * baseline (Sec. III-C, Observation I).
 *
 * The LBVH reference (Morton codes, stable sort, radix tree) gives the topology that
 * the GPU build must reproduce bit for bit; its tree is the plain top-down definition
 * (split each key range where the highest differing key bit changes).
 *
 * The last section is a CPU model of the method itself (rounds of k-buffer hit
 * collection over that tree, resuming from checkpoints), pinned against the brute-force
 * render and the paper's walkthrough; the GPU path is never compared with it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_MEM 2

/* ------------------------------------------------------------------------------------ */
/* Small linear algebra                                                                  */
/* ------------------------------------------------------------------------------------ */

static void quat_to_rot(const double qf[4], double R[3][3]) {
  double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
  double n = sqrt(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

static double quad_form(const double M[3][3], const double a[3], const double b[3]) {
  double s = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s += a[i] * M[i][j] * b[j];
  return s;
}

/* ------------------------------------------------------------------------------------ */
/* Real spherical harmonics (orthonormal, Condon-Shortley phase), from the definition    */
/* Y_l^m = sqrt(2) K_l^|m| P_l^|m|(cos th) {cos(m ph) | sin(|m| ph)}, K from factorials. */
/* ------------------------------------------------------------------------------------ */

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

/* Associated Legendre P_l^m(x), m >= 0, with the (-1)^m phase. */
static double legendre_p(int l, int m, double x) {
  double pmm = 1.0;
  if (m > 0) {
    double somx2 = sqrt((1.0 - x) * (1.0 + x));
    double fact = 1.0;
    for (int i = 1; i <= m; ++i) {
      pmm *= -fact * somx2;
      fact += 2.0;
    }
  }
  if (l == m) return pmm;
  double pmmp1 = x * (2 * m + 1) * pmm;
  if (l == m + 1) return pmmp1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m);
    pmm = pmmp1;
    pmmp1 = pll;
  }
  return pll;
}

double oracle_sh_basis(int l, int m, const double dir[3]) {
  double r = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  double x = dir[0] / r, y = dir[1] / r, z = dir[2] / r;
  double ct = z;
  double ph = atan2(y, x);
  int am = m < 0 ? -m : m;
  double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
  double P = legendre_p(l, am, ct);
  if (m == 0) return K * P;
  if (m > 0) return sqrt(2.0) * K * cos(m * ph) * P;
  return sqrt(2.0) * K * sin(am * ph) * P;
}

/* ------------------------------------------------------------------------------------ */
/* Per-Gaussian preparation                                                              */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  double mu[3];
  double sinv[3][3]; /* Sigma^-1 = R S^-2 R^T */
  double rho2;       /* 2 ln(o / alpha_min) */
  double opacity;
  int active;
  double *tri;       /* proxy mode: 20 triangles x 3 vertices x 3, world space */
} og_t;

typedef struct {
  const double *means, *scales, *quats, *opac, *sh;
  int64_t n;
  int sh_degree;
} scene_t;

/* Regular icosahedron with inradius 1: vertices (0,+-1,+-phi) and cyclic permutations,
 * faces = vertex triples at pairwise distance 2 (the edge length), wound outward, then
 * scaled so that every face plane is at distance 1 from the centre. */
static int g_ico_ready = 0;
static double g_ico_v[12][3];
static int g_ico_f[20][3];
static pthread_mutex_t g_ico_lock = PTHREAD_MUTEX_INITIALIZER;

static void ico_init(void) {
  pthread_mutex_lock(&g_ico_lock);
  if (g_ico_ready) { pthread_mutex_unlock(&g_ico_lock); return; }
  const double phi = (1.0 + sqrt(5.0)) / 2.0;
  int nv = 0;
  for (int a = -1; a <= 1; a += 2)
    for (int b = -1; b <= 1; b += 2) {
      double p[3][3] = {{0, a * 1.0, b * phi}, {a * 1.0, b * phi, 0}, {b * phi, 0, a * 1.0}};
      for (int c = 0; c < 3; ++c) {
        g_ico_v[nv][0] = p[c][0]; g_ico_v[nv][1] = p[c][1]; g_ico_v[nv][2] = p[c][2];
        ++nv;
      }
    }
  int nf = 0;
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      for (int k = j + 1; k < 12; ++k) {
        int idx[3] = {i, j, k};
        int ok = 1;
        for (int e = 0; e < 3 && ok; ++e) {
          const double *p = g_ico_v[idx[e]], *q = g_ico_v[idx[(e + 1) % 3]];
          double d2 = (p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]);
          if (fabs(d2 - 4.0) > 1e-9) ok = 0;
        }
        if (!ok) continue;
        const double *A = g_ico_v[i], *B = g_ico_v[j], *C = g_ico_v[k];
        double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double cen = nrm[0] * (A[0] + B[0] + C[0]) + nrm[1] * (A[1] + B[1] + C[1]) + nrm[2] * (A[2] + B[2] + C[2]);
        if (cen > 0) { g_ico_f[nf][0] = i; g_ico_f[nf][1] = j; g_ico_f[nf][2] = k; }
        else { g_ico_f[nf][0] = i; g_ico_f[nf][1] = k; g_ico_f[nf][2] = j; }
        ++nf;
      }
  /* inradius: distance from the centre to the plane of a face */
  const double *A = g_ico_v[g_ico_f[0][0]], *B = g_ico_v[g_ico_f[0][1]], *C = g_ico_v[g_ico_f[0][2]];
  double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double nl = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  double rin = (nrm[0] * A[0] + nrm[1] * A[1] + nrm[2] * A[2]) / nl;
  for (int v = 0; v < 12; ++v)
    for (int c = 0; c < 3; ++c) g_ico_v[v][c] /= rin;
  (void)nf;
  g_ico_ready = 1;
  pthread_mutex_unlock(&g_ico_lock);
}

int oracle_icosahedron(double *verts /* 12x3 */, int32_t *faces /* 20x3 */) {
  ico_init();
  memcpy(verts, g_ico_v, sizeof g_ico_v);
  for (int f = 0; f < 20; ++f)
    for (int c = 0; c < 3; ++c) faces[f * 3 + c] = g_ico_f[f][c];
  return OR_OK;
}

static void prepare_one(const scene_t *s, int64_t i, double alpha_min, int proxy, og_t *g) {
  double R[3][3];
  quat_to_rot(s->quats + 4 * i, R);
  double sc[3] = {s->scales[3 * i], s->scales[3 * i + 1], s->scales[3 * i + 2]};
  for (int a = 0; a < 3; ++a) g->mu[a] = s->means[3 * i + a];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += R[a][k] * R[b][k] / (sc[k] * sc[k]);
      g->sinv[a][b] = acc;
    }
  g->opacity = s->opac[i];
  g->active = g->opacity > alpha_min;
  g->rho2 = g->active ? 2.0 * log(g->opacity / alpha_min) : 0.0;
  g->tri = NULL;
  if (proxy && g->active) {
    /* world vertex = mu + R S rho * unit-space vertex */
    double rho = sqrt(g->rho2);
    double wv[12][3];
    for (int v = 0; v < 12; ++v)
      for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += R[a][k] * sc[k] * rho * g_ico_v[v][k];
        wv[v][a] = g->mu[a] + acc;
      }
    g->tri = (double *)malloc(sizeof(double) * 20 * 9);
    for (int f = 0; f < 20; ++f)
      for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) g->tri[f * 9 + c * 3 + a] = wv[g_ico_f[f][c]][a];
  }
}

/* ------------------------------------------------------------------------------------ */
/* Ray / Gaussian                                                                        */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  double t;       /* sort key distance */
  int64_t id;
  double alpha;
  double talpha;
} hit_t;

/* Ellipsoid entry: smallest root of (o + t d - mu)^T Sigma^-1 (o + t d - mu) = rho^2. */
static int ellipsoid_entry(const og_t *g, const double o[3], const double d[3], double t_near, double *t0) {
  if (!g->active) return 0;
  double f[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]};
  double A = quad_form(g->sinv, d, d);
  double B = quad_form(g->sinv, f, d);
  double C = quad_form(g->sinv, f, f) - g->rho2;
  double disc = B * B - A * C;
  if (!(disc >= 0.0)) return 0;
  double t = (-B - sqrt(disc)) / A;
  if (!(t > t_near)) return 0;
  *t0 = t;
  return 1;
}

/* Eq. 2: alpha at the point of maximum response along the ray. */
static void max_response(const og_t *g, const double o[3], const double d[3], double *alpha, double *talpha) {
  double mo[3] = {g->mu[0] - o[0], g->mu[1] - o[1], g->mu[2] - o[2]};
  double ta = quad_form(g->sinv, mo, d) / quad_form(g->sinv, d, d);
  double x[3] = {o[0] + ta * d[0] - g->mu[0], o[1] + ta * d[1] - g->mu[1], o[2] + ta * d[2] - g->mu[2]};
  double G = exp(-0.5 * quad_form(g->sinv, x, x));
  *alpha = g->opacity * G;
  *talpha = ta;
}

/* Smallest t > t_near among the front-facing icosahedron faces the ray crosses. */
static int proxy_entry(const og_t *g, const double o[3], const double d[3], double t_near, double *tp) {
  if (!g->tri) return 0;
  int found = 0;
  double best = 0.0;
  for (int f = 0; f < 20; ++f) {
    const double *A = g->tri + f * 9, *B = A + 3, *C = A + 6;
    double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double dn = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    if (!(dn < 0.0)) continue; /* back-facing or parallel */
    /* Moller-Trumbore */
    double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    double inv = 1.0 / det;
    double s[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
    if (u < 0.0 || u > 1.0) continue;
    double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    if (v < 0.0 || u + v > 1.0) continue;
    double t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    if (!(t > t_near)) continue;
    if (!found || t < best) { best = t; found = 1; }
  }
  if (found) *tp = best;
  return found;
}

/* Sphere validity of a proxy hit: the line meets the bounding ellipsoid. */
static int line_meets_ellipsoid(const og_t *g, const double o[3], const double d[3]) {
  if (!g->active) return 0;
  double f[3] = {o[0] - g->mu[0], o[1] - g->mu[1], o[2] - g->mu[2]};
  double A = quad_form(g->sinv, d, d);
  double B = quad_form(g->sinv, f, d);
  double C = quad_form(g->sinv, f, f) - g->rho2;
  return B * B - A * C >= 0.0;
}

static void sh_colour(const scene_t *s, int64_t i, const double d[3], double out[3]) {
  int K = (s->sh_degree + 1) * (s->sh_degree + 1);
  const double *c = s->sh + (size_t)i * K * 3;
  double acc[3] = {0.5, 0.5, 0.5};
  for (int l = 0; l <= s->sh_degree; ++l)
    for (int m = -l; m <= l; ++m) {
      double Y = oracle_sh_basis(l, m, d);
      int j = l * l + l + m;
      for (int ch = 0; ch < 3; ++ch) acc[ch] += Y * c[j * 3 + ch];
    }
  for (int ch = 0; ch < 3; ++ch) out[ch] = acc[ch] > 0.0 ? acc[ch] : 0.0;
}

static int hit_cmp(const void *a, const void *b) {
  const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
  if (x->t < y->t) return -1;
  if (x->t > y->t) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* ------------------------------------------------------------------------------------ */
/* Render                                                                                */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  double alpha_min, T_min, t_near;
  double bg[3];
  int key_mode; /* 0: ellipsoid entry; 1: icosahedron entry */
} params_t;

typedef struct {
  const scene_t *s;
  const og_t *g;
  const params_t *p;
  const double *ro, *rd;
  int64_t r0, r1;
  double *rgb, *depth, *opac;
  int32_t *nblend, *nhits;
  int32_t *ids; double *tafter; double *tkey; int cap;
  const double *tfar, *trans0; /* per ray, may be NULL: unbounded, T starts at 1 */
} job_t;

static void render_one(const job_t *J, int64_t r, hit_t **buf, size_t *bufcap) {
  const scene_t *s = J->s;
  const params_t *p = J->p;
  double o[3] = {J->ro[3 * r], J->ro[3 * r + 1], J->ro[3 * r + 2]};
  double d[3] = {J->rd[3 * r], J->rd[3 * r + 1], J->rd[3 * r + 2]};
  const double tfar = J->tfar ? J->tfar[r] : INFINITY;
  size_t nh = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    const og_t *g = J->g + i;
    double key;
    if (p->key_mode == 0) {
      if (!ellipsoid_entry(g, o, d, p->t_near, &key)) continue;
    } else {
      if (!proxy_entry(g, o, d, p->t_near, &key)) continue;
      if (!line_meets_ellipsoid(g, o, d)) continue;
    }
    if (!(key < tfar)) continue; /* beyond the surface that ends the ray */
    if (nh == *bufcap) {
      *bufcap = *bufcap ? 2 * *bufcap : 256;
      *buf = (hit_t *)realloc(*buf, *bufcap * sizeof(hit_t));
    }
    hit_t *h = *buf + nh++;
    h->t = key;
    h->id = i;
    max_response(g, o, d, &h->alpha, &h->talpha);
  }
  if (nh > 1) qsort(*buf, nh, sizeof(hit_t), hit_cmp); /* qsort's array may not be NULL */
  double T = J->trans0 ? J->trans0[r] : 1.0, C[3] = {0, 0, 0}, D = 0.0;
  int nb = 0;
  for (size_t h = 0; h < nh; ++h) {
    const hit_t *x = *buf + h;
    double c[3];
    sh_colour(s, x->id, d, c);
    double w = T * x->alpha;
    for (int ch = 0; ch < 3; ++ch) C[ch] += w * c[ch];
    D += w * x->talpha;
    T *= (1.0 - x->alpha);
    if (nb < J->cap) {
      if (J->ids) J->ids[r * J->cap + nb] = (int32_t)x->id;
      if (J->tafter) J->tafter[r * J->cap + nb] = T;
      if (J->tkey) J->tkey[r * J->cap + nb] = x->t;
    }
    ++nb;
    if (T < p->T_min) break;
  }
  /* the background shows only through rays that no surface ends */
  const double bgw = isinf(tfar) ? T : 0.0;
  for (int ch = 0; ch < 3; ++ch) J->rgb[3 * r + ch] = C[ch] + bgw * p->bg[ch];
  J->depth[r] = D;
  J->opac[r] = 1.0 - T;
  if (J->nblend) J->nblend[r] = nb;
  if (J->nhits) J->nhits[r] = (int32_t)nh;
}

static void *render_worker(void *arg) {
  job_t *J = (job_t *)arg;
  hit_t *buf = NULL;
  size_t cap = 0;
  for (int64_t r = J->r0; r < J->r1; ++r) render_one(J, r, &buf, &cap);
  free(buf);
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

static og_t *prepare_all(const scene_t *s, double alpha_min, int proxy) {
  if (proxy) ico_init();
  og_t *g = (og_t *)malloc(sizeof(og_t) * (size_t)(s->n > 0 ? s->n : 1));
  if (!g) return NULL;
  for (int64_t i = 0; i < s->n; ++i) prepare_one(s, i, alpha_min, proxy, g + i);
  return g;
}

static void free_all(og_t *g, int64_t n) {
  if (!g) return;
  for (int64_t i = 0; i < n; ++i) free(g[i].tri);
  free(g);
}

/* Render R rays against all Gaussians in FP64 (inputs are FP64; the tests pass float32
 * values widened exactly, or FP64 values for finite differences).
 * t_far [R] (may be NULL = unbounded): hits need key < t_far and a bounded ray gets no
 * background. trans0 [R] (may be NULL = 1): transmittance the ray starts with.
 * Outputs per ray: rgb[3], depth, opacity (1 - T); optionally the number of blended
 * hits, the number of hits, and for the first `cap` blended hits their ids, the
 * transmittance after each and the sort-key distance. */
int oracle_render(const double *means, const double *scales, const double *quats, const double *opac,
                  const double *sh, int64_t n, int sh_degree,
                  int64_t nrays, const double *ray_o, const double *ray_d,
                  const double *t_far, const double *trans0,
                  double alpha_min, double T_min, double t_near, const double *bg, int key_mode,
                  double *rgb, double *depth, double *opacity, int32_t *nblend, int32_t *nhits,
                  int32_t *ids, double *tafter, double *tkey, int cap, int nthreads) {
  if (n < 0 || nrays < 0 || sh_degree < 0 || sh_degree > 3 || !rgb || !depth || !opacity) return OR_ERR_ARG;
  if (nrays == 0) return OR_OK;
  scene_t s = {means, scales, quats, opac, sh, n, sh_degree};
  params_t p = {alpha_min, T_min, t_near, {bg ? bg[0] : 0, bg ? bg[1] : 0, bg ? bg[2] : 0}, key_mode};
  og_t *g = prepare_all(&s, alpha_min, key_mode == 1);
  if (!g) return OR_ERR_MEM;
  int nt = resolve_threads(nthreads);
  if (nt > nrays) nt = (int)nrays;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nt);
  job_t *jobs = (job_t *)malloc(sizeof(job_t) * nt);
  for (int t = 0; t < nt; ++t) {
    job_t J = {&s, g, &p, ray_o, ray_d, nrays * t / nt, nrays * (t + 1) / nt,
               rgb, depth, opacity, nblend, nhits, ids, tafter, tkey, ids || tafter || tkey ? cap : 0,
               t_far, trans0};
    jobs[t] = J;
    pthread_create(&th[t], NULL, render_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free_all(g, n);
  return OR_OK;
}

/* All hits of one ray with key in (t_near, t_far), sorted by (key, id): ids, key
 * distance, alpha, t_alpha. Returns the number of hits (entries beyond `cap` are not
 * written). */
int64_t oracle_ray_hits(const double *means, const double *scales, const double *quats, const double *opac,
                        int64_t n, const double *ray_o, const double *ray_d, double alpha_min, double t_near,
                        double t_far, int key_mode, int64_t *ids, double *tkey, double *alpha, double *talpha,
                        int64_t cap) {
  scene_t s = {means, scales, quats, opac, NULL, n, 0};
  og_t *g = prepare_all(&s, alpha_min, key_mode == 1);
  if (!g) return -1;
  double o[3] = {ray_o[0], ray_o[1], ray_o[2]}, d[3] = {ray_d[0], ray_d[1], ray_d[2]};
  hit_t *buf = (hit_t *)malloc(sizeof(hit_t) * (size_t)(n > 0 ? n : 1));
  int64_t nh = 0;
  for (int64_t i = 0; i < n; ++i) {
    double key;
    if (key_mode == 0) {
      if (!ellipsoid_entry(g + i, o, d, t_near, &key)) continue;
    } else {
      if (!proxy_entry(g + i, o, d, t_near, &key)) continue;
      if (!line_meets_ellipsoid(g + i, o, d)) continue;
    }
    if (!(key < t_far)) continue;
    buf[nh].t = key;
    buf[nh].id = i;
    max_response(g + i, o, d, &buf[nh].alpha, &buf[nh].talpha);
    ++nh;
  }
  if (nh > 1) qsort(buf, (size_t)nh, sizeof(hit_t), hit_cmp);
  for (int64_t h = 0; h < nh && h < cap; ++h) {
    if (ids) ids[h] = buf[h].id;
    if (tkey) tkey[h] = buf[h].t;
    if (alpha) alpha[h] = buf[h].alpha;
    if (talpha) talpha[h] = buf[h].talpha;
  }
  free(buf);
  free_all(g, n);
  return nh;
}

/* Composite a given ordered id list along one ray (Eq. 1 with Eq. 2 alphas), without
 * any hit test and without early termination, starting from transmittance trans0. */
int oracle_composite_list(const double *means, const double *scales, const double *quats, const double *opac,
                          const double *sh, int64_t n, int sh_degree, const double *ray_o, const double *ray_d,
                          const int32_t *list, int64_t len, double alpha_min, double trans0, const double *bg,
                          double *rgb, double *depth, double *opacity) {
  scene_t s = {means, scales, quats, opac, sh, n, sh_degree};
  double o[3] = {ray_o[0], ray_o[1], ray_o[2]}, d[3] = {ray_d[0], ray_d[1], ray_d[2]};
  double T = trans0, C[3] = {0, 0, 0}, D = 0.0;
  for (int64_t h = 0; h < len; ++h) {
    int64_t i = list[h];
    if (i < 0 || i >= n) return OR_ERR_ARG;
    og_t g;
    prepare_one(&s, i, alpha_min, 0, &g);
    double a, ta, c[3];
    max_response(&g, o, d, &a, &ta);
    sh_colour(&s, i, d, c);
    double w = T * a;
    for (int ch = 0; ch < 3; ++ch) C[ch] += w * c[ch];
    D += w * ta;
    T *= (1.0 - a);
  }
  for (int ch = 0; ch < 3; ++ch) rgb[ch] = C[ch] + T * (bg ? bg[ch] : 0.0);
  *depth = D;
  *opacity = 1.0 - T;
  return OR_OK;
}

/* Axis-aligned bounds of each Gaussian's bounding ellipsoid:
 * half-extent along axis j = sqrt(e_j^T Sigma e_j) * rho. Inactive Gaussians get
 * lo = hi = mu and active = 0. */
int oracle_gaussian_aabb(const double *means, const double *scales, const double *quats, const double *opac,
                         int64_t n, double alpha_min, double *lo, double *hi, int32_t *active) {
  for (int64_t i = 0; i < n; ++i) {
    double R[3][3];
    quat_to_rot(quats + 4 * i, R);
    double o = opac[i];
    int act = o > alpha_min;
    double rho = act ? sqrt(2.0 * log(o / alpha_min)) : 0.0;
    for (int j = 0; j < 3; ++j) {
      double var = 0.0; /* Sigma_jj */
      for (int k = 0; k < 3; ++k) var += R[j][k] * R[j][k] * (double)scales[3 * i + k] * (double)scales[3 * i + k];
      double h = act ? rho * sqrt(var) : 0.0;
      lo[3 * i + j] = (double)means[3 * i + j] - h;
      hi[3 * i + j] = (double)means[3 * i + j] + h;
    }
    active[i] = act;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Pinhole camera                                                                         */
/* ------------------------------------------------------------------------------------ */

/* Forward f = normalise(target - eye), right = normalise(f x up), true up = right x f.
 * Pixel (x, y), row 0 at the top, is sampled at its centre (x + 1/2, y + 1/2):
 * direction = normalise(f + sx * tan(fov/2) * aspect * right + sy * tan(fov/2) * up) with
 * sx = 2(x + 1/2)/W - 1, sy = 1 - 2(y + 1/2)/H, aspect = W/H, fov vertical. */
int oracle_pinhole_rays(const double *eye, const double *target, const double *up, double fov_y_deg,
                        int width, int height, double *origins, double *dirs) {
  if (width <= 0 || height <= 0) return OR_ERR_ARG;
  double f[3] = {target[0] - eye[0], target[1] - eye[1], target[2] - eye[2]};
  double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (int a = 0; a < 3; ++a) f[a] /= fl;
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (int a = 0; a < 3; ++a) r[a] /= rl;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  double th = tan(0.5 * fov_y_deg * M_PI / 180.0);
  double aspect = (double)width / (double)height;
  for (int y = 0; y < height; ++y)
    for (int x = 0; x < width; ++x) {
      int64_t i = (int64_t)y * width + x;
      double sx = (2.0 * (x + 0.5) / width - 1.0) * th * aspect;
      double sy = (1.0 - 2.0 * (y + 0.5) / height) * th;
      double d[3] = {f[0] + sx * r[0] + sy * u[0], f[1] + sx * r[1] + sy * u[1], f[2] + sx * r[2] + sy * u[2]};
      double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int a = 0; a < 3; ++a) {
        origins[3 * i + a] = eye[a];
        dirs[3 * i + a] = d[a] / dl;
      }
    }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Secondary rays: a refracting glass sphere and a reflecting rectangular mirror         */
/* ------------------------------------------------------------------------------------ */
/*
 * A ray tracer follows light past a surface by casting a new ray from the intersection
 * point (Sec. II-A); the paper's secondary-ray experiment adds a glass sphere and a
 * rectangular mirror to each scene and traces the rays they spawn (Sec. VI). Reading:
 *   - a ray ends at its first object surface beyond t_near + eps: it blends the
 *     Gaussians whose key is below that distance t_far, and what lies beyond comes from
 *     the continuation ray, which starts with the transmittance the first segment left;
 *   - mirror: the parallelogram m + x u + y v, |x| <= 1, |y| <= 1 (u, v orthogonal),
 *     two-sided, perfect reflection d - 2 (d.n) n;
 *   - glass sphere (centre c, radius r, relative index ior): solid, so no Gaussian
 *     inside it is seen; the ray refracts in by Snell's law, crosses along a chord and
 *     refracts out; total internal reflection sends it along another chord, and after
 *     OR_MAX_INSIDE chords the ray ends without a continuation;
 *   - all light follows the one continuation ray (no Fresnel split, no absorption);
 *   - eps keeps a continuation ray from meeting the surface it starts on again.
 * kind per ray: 0 no object, 1 mirror, 2 glass, 3 glass without a way out.
 */
#define OR_MAX_INSIDE 8

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Both roots of |o + t d - c|^2 = r^2 (t0 <= t1); 0 when the line misses the sphere. */
static int sphere_roots(const double c[3], double r, const double o[3], const double d[3], double *t0,
                        double *t1) {
  double f[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
  double a = dot3(d, d), b = dot3(f, d), cc = dot3(f, f) - r * r;
  double disc = b * b - a * cc;
  if (!(disc >= 0.0)) return 0;
  double sq = sqrt(disc);
  *t0 = (-b - sq) / a;
  *t1 = (-b + sq) / a;
  return 1;
}

/* Snell's law, n1 sin(theta1) = n2 sin(theta2), with the refracted ray in the plane of
 * incidence: unit d meets a surface whose unit normal n faces the ray (d.n < 0); eta =
 * n1/n2. Returns 0 on total internal reflection. */
static int refract_dir(const double d[3], const double n[3], double eta, double out[3]) {
  double ci = -dot3(d, n);
  double k = 1.0 - eta * eta * (1.0 - ci * ci);
  if (k < 0.0) return 0;
  double s = eta * ci - sqrt(k);
  for (int a = 0; a < 3; ++a) out[a] = eta * d[a] + s * n[a];
  return 1;
}

static void reflect_dir(const double d[3], const double n[3], double out[3]) {
  double dn = dot3(d, n);
  for (int a = 0; a < 3; ++a) out[a] = d[a] - 2.0 * dn * n[a];
}

/* Distance to the mirror parallelogram beyond tmin, and its unit normal. */
static int mirror_hit(const double *mir, const double o[3], const double d[3], double tmin, double *t,
                      double n[3]) {
  const double *m = mir, *u = mir + 3, *v = mir + 6;
  double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  double cl = sqrt(dot3(c, c));
  if (!(cl > 0.0)) return 0;
  for (int a = 0; a < 3; ++a) n[a] = c[a] / cl;
  double dn = dot3(d, n);
  if (dn == 0.0) return 0;
  double mo[3] = {m[0] - o[0], m[1] - o[1], m[2] - o[2]};
  double th = dot3(mo, n) / dn;
  if (!(th > tmin)) return 0;
  double q[3] = {o[0] + th * d[0] - m[0], o[1] + th * d[1] - m[1], o[2] + th * d[2] - m[2]};
  double x = dot3(q, u) / dot3(u, u), y = dot3(q, v) / dot3(v, v);
  if (!(fabs(x) <= 1.0 && fabs(y) <= 1.0)) return 0;
  *t = th;
  return 1;
}

/* Per ray: t_far (distance to the first object surface beyond t_near + eps, or +inf),
 * the continuation ray (origin, unit direction; zero when there is none), the length of
 * the bent path from the ray origin to the continuation origin, and the kind.
 * sphere = (cx, cy, cz, r, ior) or NULL; mirror = (m, u, v) or NULL. */
int oracle_object_rays(const double *sphere, const double *mirror, double eps, int64_t nrays, const double *ray_o,
                       const double *ray_d, double t_near, double *t_far, double *next_o, double *next_d,
                       double *path, int32_t *kind) {
  if (nrays < 0 || !t_far || !next_o || !next_d || !path || !kind) return OR_ERR_ARG;
  const int has_sphere = sphere && sphere[3] > 0.0;
  for (int64_t r = 0; r < nrays; ++r) {
    const double o[3] = {ray_o[3 * r], ray_o[3 * r + 1], ray_o[3 * r + 2]};
    const double d[3] = {ray_d[3 * r], ray_d[3 * r + 1], ray_d[3 * r + 2]};
    const double tmin = t_near + eps;
    double ts = INFINITY, tm = INFINITY, t0, t1, nm[3];
    if (has_sphere && sphere_roots(sphere, sphere[3], o, d, &t0, &t1)) ts = t0 > tmin ? t0 : t1 > tmin ? t1 : INFINITY;
    if (mirror && !mirror_hit(mirror, o, d, tmin, &tm, nm)) tm = INFINITY;
    double *no = next_o + 3 * r, *nd = next_d + 3 * r;
    for (int a = 0; a < 3; ++a) no[a] = nd[a] = 0.0;
    path[r] = 0.0;
    kind[r] = 0;
    t_far[r] = INFINITY;
    if (isinf(ts) && isinf(tm)) continue;
    if (tm < ts) {
      for (int a = 0; a < 3; ++a) no[a] = o[a] + tm * d[a];
      reflect_dir(d, nm, nd);
      t_far[r] = path[r] = tm;
      kind[r] = 1;
      continue;
    }
    const double *c = sphere;
    const double rad = sphere[3], ior = sphere[4];
    double p[3], dir[3] = {d[0], d[1], d[2]}, len = ts, n[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + ts * d[a];
    for (int a = 0; a < 3; ++a) n[a] = (p[a] - c[a]) / rad;
    t_far[r] = ts;
    kind[r] = 3;
    if (dot3(dir, n) < 0.0) {
      /* entering from outside: refract in (or reflect away when ior < 1 forbids entry) */
      double in[3];
      if (!refract_dir(dir, n, 1.0 / ior, in)) {
        for (int a = 0; a < 3; ++a) no[a] = p[a];
        reflect_dir(dir, n, nd);
        path[r] = len;
        kind[r] = 2;
        continue;
      }
      for (int a = 0; a < 3; ++a) dir[a] = in[a];
      if (!sphere_roots(c, rad, p, dir, &t0, &t1)) t1 = 0.0;
      len += t1;
      for (int a = 0; a < 3; ++a) p[a] += t1 * dir[a];
    }
    /* at the surface from inside: refract out, or reflect along another chord */
    for (int seg = 0; seg < OR_MAX_INSIDE; ++seg) {
      double nout[3], nin[3], out[3];
      for (int a = 0; a < 3; ++a) nout[a] = (p[a] - c[a]) / rad;
      for (int a = 0; a < 3; ++a) nin[a] = -nout[a];
      if (refract_dir(dir, nin, ior, out)) {
        for (int a = 0; a < 3; ++a) no[a] = p[a];
        for (int a = 0; a < 3; ++a) nd[a] = out[a];
        kind[r] = 2;
        break;
      }
      reflect_dir(dir, nout, out);
      for (int a = 0; a < 3; ++a) dir[a] = out[a];
      if (!sphere_roots(c, rad, p, dir, &t0, &t1)) t1 = 0.0;
      len += t1;
      for (int a = 0; a < 3; ++a) p[a] += t1 * dir[a];
    }
    path[r] = len;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* LBVH reference: Morton codes, stable sort, radix tree                                 */
/* ------------------------------------------------------------------------------------ */

/* 63-bit Morton code of each mean. The quantisation is defined in binary32 arithmetic
 * (each operation rounded to nearest float), so that it is an exact integer function of
 * the float inputs:
 *   lo_j = min_i mu_ij, hi_j = max_i mu_ij, ext_j = hi_j - lo_j,
 *   scale_j = 2^21 / ext_j (0 if ext_j == 0),
 *   q_j = clamp(floor((mu_j - lo_j) * scale_j), 0, 2^21 - 1),
 * and bit 3b+2 / 3b+1 / 3b of the code is bit b of q_x / q_y / q_z. */
int oracle_morton(int64_t n, const float *means, uint64_t *codes) {
  if (n <= 0) return OR_OK;
  volatile float lo[3], hi[3];
  for (int j = 0; j < 3; ++j) { lo[j] = means[j]; hi[j] = means[j]; }
  for (int64_t i = 1; i < n; ++i)
    for (int j = 0; j < 3; ++j) {
      float v = means[3 * i + j];
      if (v < lo[j]) lo[j] = v;
      if (v > hi[j]) hi[j] = v;
    }
  volatile float scale[3];
  for (int j = 0; j < 3; ++j) {
    volatile float ext = hi[j] - lo[j];
    scale[j] = ext > 0.0f ? 2097152.0f / ext : 0.0f;
  }
  for (int64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int j = 0; j < 3; ++j) {
      volatile float rel = means[3 * i + j] - lo[j];
      volatile float pos = rel * scale[j];
      float fl = floorf(pos);
      uint32_t v = fl <= 0.0f ? 0u : (fl >= 2097151.0f ? 2097151u : (uint32_t)fl);
      q[j] = v;
    }
    uint64_t c = 0;
    for (int b = 0; b < 21; ++b) {
      c |= (uint64_t)((q[0] >> b) & 1u) << (3 * b + 2);
      c |= (uint64_t)((q[1] >> b) & 1u) << (3 * b + 1);
      c |= (uint64_t)((q[2] >> b) & 1u) << (3 * b);
    }
    codes[i] = c;
  }
  return OR_OK;
}

static __thread const uint64_t *g_sort_codes;
static int idx_cmp(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  uint64_t cx = g_sort_codes[x], cy = g_sort_codes[y];
  if (cx != cy) return cx < cy ? -1 : 1;
  return (x > y) - (x < y);
}

typedef struct {
  const uint64_t *code; /* sorted */
  uint32_t *child;      /* [(n-1)*2] */
  uint32_t *parent;     /* [2n-1]: internal nodes first, then leaves */
  int64_t n;
} tree_t;

#define LEAF_FLAG 0x80000000u

/* Key of sorted position i: (code_i, i) as one 95-bit number. Index of the highest
 * bit in which the keys of positions a and b differ, counted from the top (0 = the
 * code's bit 62); a larger value means a longer common prefix. */
static int common_prefix(const tree_t *T, int64_t a, int64_t b) {
  uint64_t x = T->code[a] ^ T->code[b];
  if (x) {
    int p = 0;
    for (int bit = 62; bit >= 0; --bit, ++p)
      if ((x >> bit) & 1u) return p;
  }
  uint32_t y = (uint32_t)a ^ (uint32_t)b;
  int p = 63;
  for (int bit = 31; bit >= 0; --bit, ++p)
    if ((y >> bit) & 1u) return p;
  return 95;
}

/* Node covering sorted positions [first, last] (first < last) has index `self`. Its
 * split is the last position that shares more than the range's common prefix with
 * `first`; the left child covers [first, split], the right [split+1, last]. A child
 * covering a single position is a leaf; otherwise the left child is internal node
 * `split` and the right child is internal node `split+1`.
 * The split is found either by testing every position of the range (`linear`), or by
 * bisection: along sorted keys the common prefix with `first` never grows, so the
 * positions sharing more than the range's prefix form a run starting at `first`. */
static void build_range(tree_t *T, int64_t first, int64_t last, uint32_t self, int linear) {
  int range_prefix = common_prefix(T, first, last);
  int64_t split = first;
  if (linear) {
    for (int64_t i = first; i < last; ++i)
      if (common_prefix(T, first, i) > range_prefix) split = i;
  } else {
    int64_t lo = first, hi = last - 1; /* common_prefix(first, first) = 95 > range_prefix */
    while (lo < hi) {
      int64_t mid = lo + (hi - lo + 1) / 2;
      if (common_prefix(T, first, mid) > range_prefix)
        lo = mid;
      else
        hi = mid - 1;
    }
    split = lo;
  }
  uint32_t left, right;
  if (split == first) {
    left = LEAF_FLAG | (uint32_t)split;
    T->parent[(T->n - 1) + split] = self;
  } else {
    left = (uint32_t)split;
    T->parent[split] = self;
  }
  if (split + 1 == last) {
    right = LEAF_FLAG | (uint32_t)(split + 1);
    T->parent[(T->n - 1) + split + 1] = self;
  } else {
    right = (uint32_t)(split + 1);
    T->parent[split + 1] = self;
  }
  T->child[2 * self] = left;
  T->child[2 * self + 1] = right;
  if (split != first) build_range(T, first, split, (uint32_t)split, linear);
  if (split + 1 != last) build_range(T, split + 1, last, (uint32_t)(split + 1), linear);
}

/* Sort positions by (code, original index) and build the radix tree over them.
 * Outputs: sorted codes [n], perm [n] (sorted position -> original index), child
 * [(n-1)*2] (leaf children carry bit 31 and the sorted position), parent [2n-1]
 * (entries 0..n-2 for internal nodes, n-1+p for leaf p; the root's parent is
 * 0xFFFFFFFF). With `linear` every split is found by testing each position of its
 * range (quadratic in the worst case; small sizes), otherwise by bisection. */
int oracle_lbvh_topology_search(int64_t n, const float *means, uint64_t *sorted_codes, uint32_t *perm,
                                uint32_t *child, uint32_t *parent, int linear) {
  if (n <= 0) return OR_OK;
  uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  if (!codes) return OR_ERR_MEM;
  oracle_morton(n, means, codes);
  for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  g_sort_codes = codes;
  qsort(perm, (size_t)n, sizeof(uint32_t), idx_cmp);
  for (int64_t i = 0; i < n; ++i) sorted_codes[i] = codes[perm[i]];
  free(codes);
  for (int64_t i = 0; i < 2 * n - 1; ++i) parent[i] = 0xFFFFFFFFu;
  if (n == 1) return OR_OK;
  tree_t T = {sorted_codes, child, parent, n};
  build_range(&T, 0, n - 1, 0, linear);
  return OR_OK;
}

int oracle_lbvh_topology(int64_t n, const float *means, uint64_t *sorted_codes, uint32_t *perm,
                         uint32_t *child, uint32_t *parent) {
  return oracle_lbvh_topology_search(n, means, sorted_codes, perm, child, parent, 0);
}

/* ------------------------------------------------------------------------------------ */
/* CPU model of the method: multi-round k-buffer traversal with checkpoints               */
/* ------------------------------------------------------------------------------------ */
/*
 * The rendering method itself, step by step on the CPU in FP64 (Sec. III-B and IV: rounds
 * of k-nearest hit collection into a k-buffer, each followed by blending, with the
 * traversal of the next round resuming from a checkpoint). It is checked against the
 * brute-force render above (the same hits must blend in the same order, with the same
 * arithmetic) and gives the per-round state the paper's walkthrough describes.
 *
 * Structure: a binary BVH, the radix tree of oracle_lbvh_topology over the Gaussians,
 * with each Gaussian's exact bounding-ellipsoid box and each internal node's box the
 * union of its children's; every box is widened by a relative 1e-9 so that rounding
 * never puts a box entry beyond the entry of the ellipsoid inside it.
 *
 * Per ray and round:
 *   - the k-buffer holds the k nearest keys (t0, id) found in the round, sorted;
 *   - t_max, the round's cull key, is +inf until the k-buffer is full. Rule KBUF_MAX:
 *     t_max is then the k-buffer's farthest key. Rule PAPER (the walkthrough of
 *     Sec. IV-B): t_max is the nearest key rejected by, or pushed out of, the full
 *     k-buffer, that is the first such key and the ones below it;
 *   - a hit beyond the full k-buffer's farthest key is rejected, and one pushed out of it
 *     by a nearer hit is evicted: both go to the eviction list;
 *   - a node whose entry distance (raised to its parent's entry, so that entries never
 *     decrease along a path) lies beyond t_max is not visited; in CHECKPOINT mode it goes
 *     to the deferred-node list with that entry;
 *   - at the end of the round the k-buffer is blended front to back (Eq. 1) with early
 *     termination.
 * CHECKPOINT: the next round first offers the evicted hits to the empty k-buffer, then
 * takes the deferred nodes in list order, each traversed depth first, nearest child
 * first; a listed node whose entry is beyond the new t_max is listed again without a
 * visit. The ray is done at early termination or when both lists are empty.
 * RESTART: every round starts at the root; subtrees that end before the last blended
 * key and keys not beyond it are skipped. The ray is done at early termination or after
 * a round whose k-buffer did not fill.
 */

#define MODEL_CHECKPOINT 0
#define MODEL_RESTART 1
#define RULE_KBUF_MAX 0
#define RULE_PAPER 1

typedef struct {
  double t;
  int64_t id;
} mkey_t;

static int mkey_lt(mkey_t a, mkey_t b) { return a.t < b.t || (a.t == b.t && a.id < b.id); }

typedef struct {
  uint32_t ref; /* internal node index, or LEAF_FLAG | sorted position */
  double t;     /* entry distance */
} ment_t;

typedef struct {
  ment_t *a;
  size_t n, cap;
} mnvec_t;

typedef struct {
  mkey_t *a;
  size_t n, cap;
} mkvec_t;

static void mn_push(mnvec_t *v, uint32_t ref, double t) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->a = (ment_t *)realloc(v->a, v->cap * sizeof(ment_t));
  }
  v->a[v->n].ref = ref;
  v->a[v->n].t = t;
  ++v->n;
}

static void mk_push(mkvec_t *v, mkey_t k) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->a = (mkey_t *)realloc(v->a, v->cap * sizeof(mkey_t));
  }
  v->a[v->n++] = k;
}

typedef struct {
  int64_t n;
  uint32_t *child;  /* [(n-1)*2] */
  uint32_t *perm;   /* sorted position -> Gaussian */
  double *lo, *hi;  /* [2n-1][3]: internal node i at i, leaf p at n-1+p */
  int64_t *first, *last; /* sorted-position range under each node, same indexing */
  uint32_t root;
} mbvh_t;

static int64_t mb_index(const mbvh_t *B, uint32_t ref) {
  return (ref & LEAF_FLAG) ? B->n - 1 + (int64_t)(ref & ~LEAF_FLAG) : (int64_t)ref;
}

/* boxes and leaf ranges of internal node i and everything below it */
static void mb_fill(mbvh_t *B, uint32_t i) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int64_t first = INT64_MAX, last = -1;
  for (int c = 0; c < 2; ++c) {
    uint32_t ch = B->child[2 * i + c];
    if (!(ch & LEAF_FLAG)) mb_fill(B, ch);
    int64_t x = mb_index(B, ch);
    for (int a = 0; a < 3; ++a) {
      if (B->lo[3 * x + a] < lo[a]) lo[a] = B->lo[3 * x + a];
      if (B->hi[3 * x + a] > hi[a]) hi[a] = B->hi[3 * x + a];
    }
    if (B->first[x] < first) first = B->first[x];
    if (B->last[x] > last) last = B->last[x];
  }
  for (int a = 0; a < 3; ++a) {
    const double pad = 1e-9 * (1.0 + fmax(fabs(lo[a]), fabs(hi[a])));
    B->lo[3 * i + a] = lo[a] - pad;
    B->hi[3 * i + a] = hi[a] + pad;
  }
  B->first[i] = first;
  B->last[i] = last;
}

static void mb_free(mbvh_t *B) {
  free(B->child);
  free(B->perm);
  free(B->lo);
  free(B->hi);
  free(B->first);
  free(B->last);
}

static int mb_build(const scene_t *s, double alpha_min, mbvh_t *B) {
  const int64_t n = s->n;
  memset(B, 0, sizeof *B);
  B->n = n;
  if (n <= 0) return OR_OK;
  float *mf = (float *)malloc(sizeof(float) * 3 * (size_t)n);
  uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  uint32_t *parent = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(2 * n - 1));
  double *glo = (double *)malloc(sizeof(double) * 3 * (size_t)n), *ghi = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  B->child = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 1 ? 2 * (n - 1) : 1));
  B->perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  B->lo = (double *)malloc(sizeof(double) * 3 * (size_t)(2 * n - 1));
  B->hi = (double *)malloc(sizeof(double) * 3 * (size_t)(2 * n - 1));
  B->first = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
  B->last = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
  int rc = OR_OK;
  if (!mf || !codes || !parent || !glo || !ghi || !act || !B->child || !B->perm || !B->lo || !B->hi || !B->first ||
      !B->last) {
    rc = OR_ERR_MEM;
    goto done;
  }
  for (int64_t i = 0; i < 3 * n; ++i) mf[i] = (float)s->means[i];
  rc = oracle_lbvh_topology(n, mf, codes, B->perm, B->child, parent);
  if (rc != OR_OK) goto done;
  oracle_gaussian_aabb(s->means, s->scales, s->quats, s->opac, n, alpha_min, glo, ghi, act);
  for (int64_t p = 0; p < n; ++p) {
    const int64_t g = B->perm[p], x = n - 1 + p;
    for (int a = 0; a < 3; ++a) {
      const double pad = 1e-9 * (1.0 + fmax(fabs(glo[3 * g + a]), fabs(ghi[3 * g + a])));
      B->lo[3 * x + a] = glo[3 * g + a] - pad;
      B->hi[3 * x + a] = ghi[3 * g + a] + pad;
    }
    B->first[x] = B->last[x] = p;
  }
  if (n == 1) {
    B->root = LEAF_FLAG;
  } else {
    B->root = 0;
    mb_fill(B, 0);
  }
done:
  free(mf);
  free(codes);
  free(parent);
  free(glo);
  free(ghi);
  free(act);
  if (rc != OR_OK) mb_free(B);
  return rc;
}

/* Slab test of box x: entry and exit distances of the line; 0 if it misses the box. */
static int mb_slab(const mbvh_t *B, int64_t x, const double o[3], const double d[3], double *tn, double *tf) {
  double a0 = -INFINITY, a1 = INFINITY;
  for (int a = 0; a < 3; ++a) {
    const double lo = B->lo[3 * x + a], hi = B->hi[3 * x + a];
    if (d[a] == 0.0) {
      if (o[a] < lo || o[a] > hi) return 0;
      continue;
    }
    double t0 = (lo - o[a]) / d[a], t1 = (hi - o[a]) / d[a];
    if (t0 > t1) {
      const double tt = t0;
      t0 = t1;
      t1 = tt;
    }
    if (t0 > a0) a0 = t0;
    if (t1 < a1) a1 = t1;
  }
  if (!(a0 <= a1)) return 0;
  *tn = a0;
  *tf = a1;
  return 1;
}

typedef struct {
  int k, mode, rule;
  double alpha_min, T_min;
} mparams_t;

typedef struct {
  double rgb[3], depth, opacity;
  int32_t nblend, rounds;
  int64_t nodes, leaves, deferred, evicted;
  int64_t unique;  /* distinct nodes and leaves visited */
  int64_t peak;    /* largest checkpoint carried between rounds: deferred nodes + evicted hits */
} mres_t;

/* end-of-round state of one round (before its blend), for one ray */
typedef struct {
  int round;
  mkvec_t kbuf, ev;
  mnvec_t def;
  mkey_t tmax;
  int logged;
} mlog_t;

typedef struct {
  const mbvh_t *B;
  const og_t *g;
  const scene_t *s;
  const mparams_t *P;
  double o[3], d[3];
  mkvec_t kbuf, esrc, edst;
  mnvec_t nsrc, ndst, stack;
  mkey_t tmax, tmin;
  mres_t *res;
  uint64_t *seen;     /* one bit per node and leaf: visited by this ray */
  uint32_t *touched;  /* words of `seen` set by this ray, cleared after it */
  size_t ntouched, touched_cap;
} mray_t;

/* count a visit of node or leaf index x (mb_index) as new or repeated */
static void m_visit(mray_t *R, int64_t x) {
  uint64_t *w = R->seen + (x >> 6);
  const uint64_t bit = 1ull << (x & 63);
  if (*w & bit) return;
  if (*w == 0) {
    if (R->ntouched == R->touched_cap) {
      R->touched_cap = R->touched_cap ? 2 * R->touched_cap : 256;
      R->touched = (uint32_t *)realloc(R->touched, R->touched_cap * sizeof(uint32_t));
    }
    R->touched[R->ntouched++] = (uint32_t)(x >> 6);
  }
  *w |= bit;
  ++R->res->unique;
}

static void m_offer(mray_t *R, mkey_t key) {
  mkvec_t *kb = &R->kbuf;
  const int k = R->P->k;
  if ((int)kb->n == k && mkey_lt(kb->a[k - 1], key)) {
    /* rejected: beyond the full k-buffer */
    if (R->P->mode == MODEL_CHECKPOINT) mk_push(&R->edst, key), ++R->res->evicted;
    if (R->P->rule == RULE_PAPER && mkey_lt(key, R->tmax)) R->tmax = key;
    return;
  }
  /* sorted insertion; a full buffer pushes out its farthest key */
  mk_push(kb, key);
  size_t j = kb->n - 1;
  while (j > 0 && mkey_lt(key, kb->a[j - 1])) {
    kb->a[j] = kb->a[j - 1];
    --j;
  }
  kb->a[j] = key;
  if ((int)kb->n > k) {
    const mkey_t out = kb->a[--kb->n];
    if (R->P->mode == MODEL_CHECKPOINT) mk_push(&R->edst, out), ++R->res->evicted;
    if (R->P->rule == RULE_PAPER && mkey_lt(out, R->tmax)) R->tmax = out;
  }
  if (R->P->rule == RULE_KBUF_MAX && (int)kb->n == k) R->tmax = kb->a[k - 1];
}

static void m_defer(mray_t *R, uint32_t ref, double t) {
  if (R->P->mode == MODEL_CHECKPOINT) {
    mn_push(&R->ndst, ref, t);
    ++R->res->deferred;
  }
}

/* depth-first traversal of the subtree at `ref` (entry distance t) */
static void m_traverse(mray_t *R, uint32_t ref, double t) {
  const mbvh_t *B = R->B;
  const int restart = R->P->mode == MODEL_RESTART;
  R->stack.n = 0;
  mn_push(&R->stack, ref, t);
  while (R->stack.n) {
    const ment_t e = R->stack.a[--R->stack.n];
    if (e.t > R->tmax.t) { /* t_max came down since the node was reached */
      m_defer(R, e.ref, e.t);
      continue;
    }
    if (R->seen) m_visit(R, mb_index(B, e.ref));
    if (e.ref & LEAF_FLAG) {
      ++R->res->leaves;
      const int64_t gid = B->perm[e.ref & ~LEAF_FLAG];
      double t0;
      if (!ellipsoid_entry(R->g + gid, R->o, R->d, 0.0, &t0)) continue;
      const mkey_t key = {t0, gid};
      if (restart && !mkey_lt(R->tmin, key)) continue; /* blended in an earlier round */
      m_offer(R, key);
      continue;
    }
    ++R->res->nodes;
    double tc[2];
    uint32_t rc[2];
    int nc = 0;
    for (int c = 0; c < 2; ++c) {
      const uint32_t ch = B->child[2 * e.ref + c];
      double tn, tf;
      if (!mb_slab(B, mb_index(B, ch), R->o, R->d, &tn, &tf)) continue;
      if (tf < 0.0) continue;                    /* behind the ray origin */
      if (restart && tf < R->tmin.t) continue;   /* ends before the last blended key */
      const double te = tn > e.t ? tn : e.t;     /* entries never decrease along a path */
      if (te > R->tmax.t) {
        m_defer(R, ch, te);
        continue;
      }
      rc[nc] = ch;
      tc[nc] = te;
      ++nc;
    }
    /* nearer child on top of the stack */
    if (nc == 2 && tc[1] > tc[0]) {
      mn_push(&R->stack, rc[1], tc[1]);
      mn_push(&R->stack, rc[0], tc[0]);
    } else {
      for (int c = 0; c < nc; ++c) mn_push(&R->stack, rc[c], tc[c]);
    }
  }
}

static void m_copy_log(mray_t *R, mlog_t *L) {
  L->kbuf.n = L->ev.n = L->def.n = 0;
  for (size_t i = 0; i < R->kbuf.n; ++i) mk_push(&L->kbuf, R->kbuf.a[i]);
  for (size_t i = 0; i < R->edst.n; ++i) mk_push(&L->ev, R->edst.a[i]);
  for (size_t i = 0; i < R->ndst.n; ++i) mn_push(&L->def, R->ndst.a[i].ref, R->ndst.a[i].t);
  L->tmax = R->tmax;
  L->logged = 1;
}

/* One ray through all its rounds. ids / round_of: the first `cap` blended hits. */
static void m_ray(mray_t *R, int cap, int32_t *ids, int32_t *round_of, mlog_t *L) {
  const mbvh_t *B = R->B;
  const mparams_t *P = R->P;
  mres_t *res = R->res;
  memset(res, 0, sizeof *res);
  R->nsrc.n = R->ndst.n = R->esrc.n = R->edst.n = R->kbuf.n = 0;
  R->tmin.t = -INFINITY;
  R->tmin.id = -1;
  double root_t = 0.0, root_f = 0.0;
  const int root_hit = B->n > 0 && mb_slab(B, mb_index(B, B->root), R->o, R->d, &root_t, &root_f) && root_f >= 0.0;
  if (root_hit) mn_push(&R->nsrc, B->root, root_t);
  double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
  int nb = 0, done = 0;
  while (!done) {
    ++res->rounds;
    R->kbuf.n = R->edst.n = R->ndst.n = 0;
    R->tmax.t = INFINITY;
    R->tmax.id = INT64_MAX;
    if (P->mode == MODEL_CHECKPOINT) {
      for (size_t i = 0; i < R->esrc.n; ++i) m_offer(R, R->esrc.a[i]);
      for (size_t i = 0; i < R->nsrc.n; ++i) {
        const ment_t e = R->nsrc.a[i];
        if (e.t > R->tmax.t)
          m_defer(R, e.ref, e.t);
        else
          m_traverse(R, e.ref, e.t);
      }
    } else if (root_hit) {
      m_traverse(R, B->root, root_t);
    }
    if (L && L->round == res->rounds) m_copy_log(R, L);
    const int full = (int)R->kbuf.n == P->k;
    int ert = 0;
    for (size_t i = 0; i < R->kbuf.n; ++i) {
      const mkey_t key = R->kbuf.a[i];
      double alpha, talpha, c[3];
      max_response(R->g + key.id, R->o, R->d, &alpha, &talpha);
      sh_colour(R->s, key.id, R->d, c);
      const double w = T * alpha;
      for (int ch = 0; ch < 3; ++ch) C[ch] += w * c[ch];
      D += w * talpha;
      T *= (1.0 - alpha);
      if (nb < cap) {
        if (ids) ids[nb] = (int32_t)key.id;
        if (round_of) round_of[nb] = res->rounds;
      }
      ++nb;
      R->tmin = key;
      if (T < P->T_min) {
        ert = 1;
        break;
      }
    }
    if ((int64_t)(R->ndst.n + R->edst.n) > res->peak) res->peak = (int64_t)(R->ndst.n + R->edst.n);
    if (ert) {
      done = 1;
    } else if (P->mode == MODEL_CHECKPOINT) {
      /* the lists of this round are the next round's sources */
      mnvec_t tn = R->nsrc;
      R->nsrc = R->ndst;
      R->ndst = tn;
      mkvec_t te = R->esrc;
      R->esrc = R->edst;
      R->edst = te;
      done = R->nsrc.n == 0 && R->esrc.n == 0;
    } else {
      done = !full;
    }
  }
  for (int ch = 0; ch < 3; ++ch) res->rgb[ch] = C[ch];
  res->depth = D;
  res->opacity = 1.0 - T;
  res->nblend = nb;
  if (R->seen)
    for (size_t i = 0; i < R->ntouched; ++i) R->seen[R->touched[i]] = 0;
  R->ntouched = 0;
}

/* per-ray visit bitmap over the 2n-1 nodes and leaves */
static int m_ray_init(mray_t *R, const mbvh_t *B) {
  const int64_t words = (2 * B->n - 1 + 63) / 64 + 1;
  R->seen = (uint64_t *)calloc((size_t)words, sizeof(uint64_t));
  return R->seen ? OR_OK : OR_ERR_MEM;
}

static void m_ray_free(mray_t *R) {
  free(R->seen);
  free(R->touched);
  free(R->kbuf.a);
  free(R->esrc.a);
  free(R->edst.a);
  free(R->nsrc.a);
  free(R->ndst.a);
  free(R->stack.a);
}

typedef struct {
  const mbvh_t *B;
  const og_t *g;
  const scene_t *s;
  const mparams_t *P;
  const double *ro, *rd;
  int64_t r0, r1;
  int cap;
  double *rgb, *depth, *opac;
  int32_t *nblend, *ids, *round_of, *rounds;
  int64_t *counts;
  int distinct;
  int failed;
} mjob_t;

static void *m_worker(void *arg) {
  mjob_t *J = (mjob_t *)arg;
  mray_t R;
  memset(&R, 0, sizeof R);
  R.B = J->B;
  R.g = J->g;
  R.s = J->s;
  R.P = J->P;
  mres_t res;
  R.res = &res;
  if (J->distinct && m_ray_init(&R, J->B) != OR_OK) {
    J->failed = 1;
    return NULL;
  }
  for (int64_t r = J->r0; r < J->r1; ++r) {
    for (int a = 0; a < 3; ++a) {
      R.o[a] = J->ro[3 * r + a];
      R.d[a] = J->rd[3 * r + a];
    }
    m_ray(&R, J->cap, J->ids ? J->ids + r * J->cap : NULL, J->round_of ? J->round_of + r * J->cap : NULL, NULL);
    for (int ch = 0; ch < 3; ++ch) J->rgb[3 * r + ch] = res.rgb[ch];
    J->depth[r] = res.depth;
    J->opac[r] = res.opacity;
    if (J->nblend) J->nblend[r] = res.nblend;
    if (J->rounds) J->rounds[r] = res.rounds;
    if (J->counts) {
      int64_t *c = J->counts + 6 * r;
      c[0] = res.nodes;
      c[1] = res.leaves;
      c[2] = res.deferred;
      c[3] = res.evicted;
      c[4] = res.unique;
      c[5] = res.peak;
    }
  }
  m_ray_free(&R);
  return NULL;
}

/* The method on the CPU for R rays (unit directions, t_near = 0, black background).
 * k >= 1; mode MODEL_CHECKPOINT or MODEL_RESTART; rule RULE_KBUF_MAX or RULE_PAPER.
 * Outputs per ray: rgb[3], depth, opacity; optionally the number of blended hits and of
 * rounds, the first `cap` blended ids and the round that blended each, and six counts
 * (internal nodes visited, leaves tested, nodes deferred, hits evicted, distinct nodes
 * and leaves visited, and the largest checkpoint carried from one round to the next in
 * entries: deferred nodes plus evicted hits; the distinct count only with `distinct`, which
 * costs a visit bitmap per thread, otherwise 0). */
int oracle_model_render(const double *means, const double *scales, const double *quats, const double *opac,
                        const double *sh, int64_t n, int sh_degree, int64_t nrays, const double *ray_o,
                        const double *ray_d, double alpha_min, double T_min, int k, int mode, int rule, int cap,
                        int nthreads, double *rgb, double *depth, double *opacity, int32_t *nblend, int32_t *ids,
                        int32_t *round_of, int32_t *rounds, int64_t *counts, int distinct) {
  if (n < 0 || nrays < 0 || k < 1 || (mode != MODEL_CHECKPOINT && mode != MODEL_RESTART) ||
      (rule != RULE_KBUF_MAX && rule != RULE_PAPER) || cap < 0)
    return OR_ERR_ARG;
  scene_t s = {means, scales, quats, opac, sh, n, sh_degree};
  mparams_t P = {k, mode, rule, alpha_min, T_min};
  mbvh_t B;
  int rc = mb_build(&s, alpha_min, &B);
  if (rc != OR_OK) return rc;
  og_t *g = prepare_all(&s, alpha_min, 0);
  if (!g) {
    mb_free(&B);
    return OR_ERR_MEM;
  }
  int nt = resolve_threads(nthreads);
  if (nt > nrays) nt = nrays > 0 ? (int)nrays : 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
  mjob_t *jobs = (mjob_t *)malloc(sizeof(mjob_t) * (size_t)nt);
  if (!th || !jobs) {
    free(th);
    free(jobs);
    free_all(g, n);
    mb_free(&B);
    return OR_ERR_MEM;
  }
  for (int t = 0; t < nt; ++t) {
    mjob_t J = {&B, g, &s, &P, ray_o, ray_d, nrays * t / nt, nrays * (t + 1) / nt, cap, rgb, depth, opacity,
                nblend, ids, round_of, rounds, counts, distinct, 0};
    jobs[t] = J;
    pthread_create(th + t, NULL, m_worker, jobs + t);
  }
  int failed = 0;
  for (int t = 0; t < nt; ++t) {
    pthread_join(th[t], NULL);
    failed |= jobs[t].failed;
  }
  free(th);
  free(jobs);
  free_all(g, n);
  mb_free(&B);
  return failed ? OR_ERR_MEM : OR_OK;
}

/* The state of one ray at the end of round `round` (1-based), before that round blends:
 * the k-buffer's keys (ids, distances), the eviction list, the deferred nodes (the range
 * of sorted leaf positions under each, as oracle_lbvh_topology orders them, and its entry
 * distance) and t_max (distance and id; +inf and INT64_MAX while the k-buffer was not
 * full). *n_* receive the full list lengths; at most the given capacities are written.
 * Returns OR_ERR_ARG when the ray finishes before that round. */
int oracle_model_round_state(const double *means, const double *scales, const double *quats, const double *opac,
                             const double *sh, int64_t n, int sh_degree, const double *ray_o, const double *ray_d,
                             double alpha_min, double T_min, int k, int mode, int rule, int round,
                             int64_t *kbuf_ids, double *kbuf_t, int32_t *n_kbuf, int64_t *ev_ids, double *ev_t,
                             int32_t *n_ev, int ev_cap, int64_t *def_first, int64_t *def_last, double *def_t,
                             int32_t *n_def, int def_cap, double *tmax_t, int64_t *tmax_id) {
  if (n < 0 || k < 1 || round < 1 || (mode != MODEL_CHECKPOINT && mode != MODEL_RESTART) ||
      (rule != RULE_KBUF_MAX && rule != RULE_PAPER))
    return OR_ERR_ARG;
  scene_t s = {means, scales, quats, opac, sh, n, sh_degree};
  mparams_t P = {k, mode, rule, alpha_min, T_min};
  mbvh_t B;
  int rc = mb_build(&s, alpha_min, &B);
  if (rc != OR_OK) return rc;
  og_t *g = prepare_all(&s, alpha_min, 0);
  if (!g) {
    mb_free(&B);
    return OR_ERR_MEM;
  }
  mray_t R;
  memset(&R, 0, sizeof R);
  mres_t res;
  R.B = &B;
  R.g = g;
  R.s = &s;
  R.P = &P;
  R.res = &res;
  if (m_ray_init(&R, &B) != OR_OK) {
    free_all(g, n);
    mb_free(&B);
    return OR_ERR_MEM;
  }
  for (int a = 0; a < 3; ++a) {
    R.o[a] = ray_o[a];
    R.d[a] = ray_d[a];
  }
  mlog_t L;
  memset(&L, 0, sizeof L);
  L.round = round;
  m_ray(&R, 0, NULL, NULL, &L);
  if (L.logged) {
    *n_kbuf = (int32_t)L.kbuf.n;
    for (size_t i = 0; i < L.kbuf.n && (int)i < k; ++i) {
      kbuf_ids[i] = L.kbuf.a[i].id;
      kbuf_t[i] = L.kbuf.a[i].t;
    }
    *n_ev = (int32_t)L.ev.n;
    for (size_t i = 0; i < L.ev.n && (int)i < ev_cap; ++i) {
      ev_ids[i] = L.ev.a[i].id;
      ev_t[i] = L.ev.a[i].t;
    }
    *n_def = (int32_t)L.def.n;
    for (size_t i = 0; i < L.def.n && (int)i < def_cap; ++i) {
      const int64_t x = mb_index(&B, L.def.a[i].ref);
      def_first[i] = B.first[x];
      def_last[i] = B.last[x];
      def_t[i] = L.def.a[i].t;
    }
    *tmax_t = L.tmax.t;
    *tmax_id = L.tmax.id;
  }
  free(L.kbuf.a);
  free(L.ev.a);
  free(L.def.a);
  m_ray_free(&R);
  free_all(g, n);
  mb_free(&B);
  return L.logged ? OR_OK : OR_ERR_ARG;
}
