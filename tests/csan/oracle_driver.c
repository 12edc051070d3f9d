/* Drives every oracle entry point on small seeded inputs, for a build of the oracle with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py).
 * Exits non-zero on a failed call; the sanitizers abort on a memory or UB error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_render(const double *means, const double *scales, const double *quats, const double *opac,
                  const double *sh, int64_t n, int sh_degree, int64_t nrays, const double *ray_o,
                  const double *ray_d, const double *t_far, const double *trans0, double alpha_min, double T_min,
                  double t_near, const double *bg, int key_mode, double *rgb, double *depth, double *opacity,
                  int32_t *nblend, int32_t *nhits, int32_t *ids, double *tafter, double *tkey, int cap, int nthreads);
int64_t oracle_ray_hits(const double *means, const double *scales, const double *quats, const double *opac,
                        int64_t n, const double *ray_o, const double *ray_d, double alpha_min, double t_near,
                        double t_far, int key_mode, int64_t *ids, double *tkey, double *alpha, double *talpha,
                        int64_t cap);
int oracle_pinhole_rays(const double *eye, const double *target, const double *up, double fov_y_deg, int width,
                        int height, double *origins, double *dirs);
int oracle_lbvh_topology(int64_t n, const float *means, uint64_t *sorted_codes, uint32_t *perm, uint32_t *child,
                         uint32_t *parent);
int oracle_icosahedron(double *verts, int32_t *faces);
int oracle_object_rays(const double *sphere, const double *mirror, double eps, int64_t nrays, const double *ray_o,
                       const double *ray_d, double t_near, double *t_far, double *next_o, double *next_d,
                       double *path, int32_t *kind);

int oracle_model_render(const double *means, const double *scales, const double *quats, const double *opac,
                        const double *sh, int64_t n, int sh_degree, int64_t nrays, const double *ray_o,
                        const double *ray_d, double alpha_min, double T_min, int k, int mode, int rule, int cap,
                        int nthreads, double *rgb, double *depth, double *opacity, int32_t *nblend, int32_t *ids,
                        int32_t *round_of, int32_t *rounds, int64_t *counts, int distinct);
int oracle_model_round_state(const double *means, const double *scales, const double *quats, const double *opac,
                             const double *sh, int64_t n, int sh_degree, const double *ray_o, const double *ray_d,
                             double alpha_min, double T_min, int k, int mode, int rule, int round,
                             int64_t *kbuf_ids, double *kbuf_t, int32_t *n_kbuf, int64_t *ev_ids, double *ev_t,
                             int32_t *n_ev, int ev_cap, int64_t *def_first, int64_t *def_last, double *def_t,
                             int32_t *n_def, int def_cap, double *tmax_t, int64_t *tmax_id);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, a plain test-input generator */
  state ^= state >> 12; state ^= state << 25; state ^= state >> 27;
  return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) / 9007199254740992.0;
}

int main(void) {
  enum { N = 200, W = 16, H = 12, CAP = 64 };
  const int R = W * H, L = 3, NC = (L + 1) * (L + 1);
  double *means = malloc(sizeof(double) * 3 * N), *scales = malloc(sizeof(double) * 3 * N);
  double *quats = malloc(sizeof(double) * 4 * N), *opac = malloc(sizeof(double) * N);
  double *sh = malloc(sizeof(double) * 3 * NC * N);
  float *fm = malloc(sizeof(float) * 3 * N);
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) {
      means[3 * i + a] = 2.0 * urand() - 1.0;
      scales[3 * i + a] = 0.02 + 0.1 * urand();
      fm[3 * i + a] = (float)means[3 * i + a];
    }
    for (int a = 0; a < 4; ++a) quats[4 * i + a] = urand() - 0.5;
    opac[i] = urand();
    for (int c = 0; c < 3 * NC; ++c) sh[3 * NC * i + c] = urand() - 0.5;
  }
  double eye[3] = {0, -3, 0}, tgt[3] = {0, 0, 0}, up[3] = {0, 0, 1};
  double *o = malloc(sizeof(double) * 3 * R), *d = malloc(sizeof(double) * 3 * R);
  if (oracle_pinhole_rays(eye, tgt, up, 60.0, W, H, o, d)) return 1;
  double *rgb = malloc(sizeof(double) * 3 * R), *dep = malloc(sizeof(double) * R), *op = malloc(sizeof(double) * R);
  int32_t *nb = malloc(sizeof(int32_t) * R), *nh = malloc(sizeof(int32_t) * R), *ids = malloc(sizeof(int32_t) * R * CAP);
  double *ta = malloc(sizeof(double) * R * CAP), *tk = malloc(sizeof(double) * R * CAP);
  for (int key_mode = 0; key_mode <= 1; ++key_mode)
    if (oracle_render(means, scales, quats, opac, sh, N, L, R, o, d, NULL, NULL, 1.0 / 255.0, 1e-3, 0.0, NULL,
                      key_mode, rgb, dep, op, nb, nh, ids, ta, tk, CAP, 4))
      return 2;
  int64_t hid[CAP];
  double hk[CAP], ha[CAP], ht[CAP];
  if (oracle_ray_hits(means, scales, quats, opac, N, o, d, 1.0 / 255.0, 0.0, 1e30, 0, hid, hk, ha, ht, CAP) < 0)
    return 3;
  /* objects, then the bounded render of the primary rays and of the continuation rays */
  double sphere[5] = {0.2, 0.0, 0.1, 0.5, 1.5};
  double mirror[9] = {-0.5, 0.3, -0.2, 0.6, 0.0, 0.2, 0.0, 0.5, 0.0};
  double *tf = malloc(sizeof(double) * R), *no = malloc(sizeof(double) * 3 * R), *nd = malloc(sizeof(double) * 3 * R);
  double *pl = malloc(sizeof(double) * R), *t0 = malloc(sizeof(double) * R);
  int32_t *kd = malloc(sizeof(int32_t) * R);
  if (oracle_object_rays(sphere, mirror, 1e-4, R, o, d, 0.0, tf, no, nd, pl, kd)) return 6;
  for (int r = 0; r < R; ++r) t0[r] = 0.5 + 0.5 * urand();
  if (oracle_render(means, scales, quats, opac, sh, N, L, R, o, d, tf, t0, 1.0 / 255.0, 1e-3, 0.0, NULL, 0, rgb,
                    dep, op, nb, nh, ids, ta, tk, CAP, 4))
    return 7;
  if (oracle_object_rays(sphere, mirror, 1e-4, R, no, nd, 0.0, tf, o, d, pl, kd)) return 8;
  free(tf); free(no); free(nd); free(pl); free(t0); free(kd);
  uint64_t *codes = malloc(sizeof(uint64_t) * N);
  uint32_t *perm = malloc(sizeof(uint32_t) * N), *child = malloc(sizeof(uint32_t) * 2 * (N - 1));
  uint32_t *parent = malloc(sizeof(uint32_t) * (2 * N - 1));
  if (oracle_lbvh_topology(N, fm, codes, perm, child, parent)) return 4;
  double v[36];
  int32_t f[60];
  if (oracle_icosahedron(v, f)) return 5;
  /* the CPU model of the method: every mode and rule, k from 1 to above the hit count,
   * on the scene and on a one-Gaussian scene; then one ray's round-2 state */
  int32_t *ro = malloc(sizeof(int32_t) * R * CAP), *nr = malloc(sizeof(int32_t) * R);
  int64_t *cnt = malloc(sizeof(int64_t) * 6 * R);
  for (int k = 1; k <= 64; k *= 4)
    for (int mode = 0; mode <= 1; ++mode)
      for (int rule = 0; rule <= 1; ++rule) {
        if (oracle_model_render(means, scales, quats, opac, sh, N, L, R, o, d, 1.0 / 255.0, 1e-3, k, mode, rule, CAP,
                                4, rgb, dep, op, nb, ids, ro, nr, cnt, rule))
          return 9;
        if (oracle_model_render(means, scales, quats, opac, sh, 1, L, R, o, d, 1.0 / 255.0, 1e-3, k, mode, rule, 0, 2,
                                rgb, dep, op, NULL, NULL, NULL, NULL, NULL, 1))
          return 10;
      }
  {
    int64_t ki[4], ei[CAP], df[CAP], dl[CAP], ti;
    double kt[4], et[CAP], dt[CAP], tt;
    int32_t nk, ne, nd;
    int best = 0;
    for (int r = 0; r < R; ++r)
      if (nb[r] > nb[best]) best = r; /* most blended hits: several rounds at k = 4 */
    (void)oracle_model_round_state(means, scales, quats, opac, sh, N, L, o + 3 * best, d + 3 * best, 1.0 / 255.0, 1e-3,
                                   4, 0, 1, 2, ki, kt, &nk, ei, et, &ne, CAP, df, dl, dt, &nd, CAP, &tt, &ti);
  }
  free(ro); free(nr); free(cnt);
  printf("ok %.6f\n", rgb[0] + dep[R / 2]);
  free(means); free(scales); free(quats); free(opac); free(sh); free(fm); free(o); free(d); free(rgb);
  free(dep); free(op); free(nb); free(nh); free(ids); free(ta); free(tk); free(codes); free(perm);
  free(child); free(parent);
  return 0;
}
