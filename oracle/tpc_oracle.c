/*
 * tpc_oracle.c -- FP64 CPU reference of the TPC sector tracker.
 *
 * TEST INFRASTRUCTURE: the oracle the GPU path is checked against.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * It follows the method of Rohr et al., "ALICE HLT TPC Tracking of Pb-Pb
 * Events on GPUs", step by step and in the paper's order:
 *   section 1, neighbours finder   -> nf_row()
 *   section 1, evolution step      -> orc_evolve()
 *   section 1, chains -> tracklets -> sector_seeds()
 *   section 1, tracklet construction (Kalman fit, extrapolation to adjacent
 *              rows, chi^2 condition, refit)            -> build_tracklet()
 *   section 1 + 3.1, tracklet selection with the cluster weight
 *              w = n (alpha - chi^2/beta)               -> select_core()
 *   section 3.2, sorted output                          -> track_sector()
 * Each sector is tracked on its own (section 1); the CPU tracker parallelises
 * trivially over sectors (section 4), and so does this file.
 *
 * Where the paper leaves a choice open (track model, windows, gates, the
 * order of fit and extension, the chi^2 normalisation), the reading used
 * here is the one documented with each function.  Nothing here is blocked,
 * fused or reordered for speed: candidate searches use a y-sorted copy of each
 * row only to avoid visiting every cluster, and apply the exact criteria.
 */
#include "tpc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define CLIGHT 0.00299792458 /* GeV / (T cm) */

void orc_params_default(orc_params* p) {
  /* The same numbers as the FP32 parameters of the GPU path, widened. */
  p->sigma_y = (double)0.1f;
  p->sigma_z = (double)0.1f;
  p->nf_win_y = 4.0;
  p->nf_win_z = 4.0;
  p->nf_chi2_max = 25.0;
  p->min_seed_len = 3;
  p->seed_window = 16;
  p->chi2_gate = 16.0;
  p->max_miss = 10;
  p->max_sinphi = (double)0.95f;
  p->alpha = 6.0; /* section 3.1: the chosen chi^2-suppression factor */
  p->beta = 1.0;
  p->min_clusters = 30; /* section 5: sector tracks have >= 30 clusters */
  p->min_pt = (double)0.1f;
  p->prior_sinphi = 1.0;
  p->prior_tanl = 1.0;
  p->prior_qpt = 100.0;
}

/* ------------------------------------------------------------------------ */
/* Sector context                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_event* ev;
  const orc_geometry* geo;
  const orc_params* prm;
  double bz;
  int slot;
  int nr;
  const int32_t* ro; /* row offsets of this sector: nr + 1 entries */
  int32_t* sorted;   /* per row, global indices sorted by (y, index) */
} sector_ctx;

typedef struct {
  double y;
  int32_t i;
} y_idx;

static int cmp_y_idx(const void* a, const void* b) {
  const y_idx* p = (const y_idx*)a;
  const y_idx* q = (const y_idx*)b;
  if (p->y < q->y) return -1;
  if (p->y > q->y) return 1;
  return (p->i > q->i) - (p->i < q->i);
}

static int sector_init(sector_ctx* sc, const orc_event* ev, const orc_geometry* geo,
                       const orc_params* prm, double bz, int slot) {
  sc->ev = ev;
  sc->geo = geo;
  sc->prm = prm;
  sc->bz = bz;
  sc->slot = slot;
  sc->nr = geo->n_rows;
  sc->ro = ev->row_offsets + (int64_t)slot * geo->n_rows;
  int64_t base = sc->ro[0], n = sc->ro[sc->nr] - base;
  sc->sorted = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  y_idx* tmp = (y_idx*)malloc(sizeof(y_idx) * (size_t)(n > 0 ? n : 1));
  if (!sc->sorted || !tmp) {
    free(sc->sorted);
    free(tmp);
    return -1;
  }
  for (int64_t i = 0; i < n; ++i) {
    tmp[i].y = ev->y[base + i];
    tmp[i].i = (int32_t)(base + i);
  }
  for (int r = 0; r < sc->nr; ++r) {
    int64_t b = sc->ro[r] - base, e = sc->ro[r + 1] - base;
    if (e - b > 1) qsort(tmp + b, (size_t)(e - b), sizeof(y_idx), cmp_y_idx);
  }
  for (int64_t i = 0; i < n; ++i) sc->sorted[i] = tmp[i].i;
  free(tmp);
  return 0;
}

static void sector_free(sector_ctx* sc) { free(sc->sorted); }

/* First position in the y-sorted row r whose y is >= ylo. */
static int64_t row_lower_bound(const sector_ctx* sc, int r, double ylo) {
  int64_t base = sc->ro[0];
  int64_t lo = sc->ro[r] - base, hi = sc->ro[r + 1] - base;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if ((double)sc->ev->y[sc->sorted[mid]] < ylo)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

static int row_of_cluster(const sector_ctx* sc, int32_t c) {
  int lo = 0, hi = sc->nr - 1; /* find r with ro[r] <= c < ro[r+1] */
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (sc->ro[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

/* ------------------------------------------------------------------------ */
/* Neighbours finder (section 1, first combinatorial step)                  */
/* ------------------------------------------------------------------------ */
/*
 * For a cluster c on row k the paper looks for the best pair of neighbours on
 * rows k-1 and k+1 that forms a straight line with c, and stores both links.
 * Reading used: candidates lie inside a window |dy| <= nf_win_y, |dz| <=
 * nf_win_z around c on each neighbour row; the straightness measure is the
 * residual of c from the chord d-u at x_k, normalised by its variance for
 * three clusters of resolution sigma:
 *   t = (x_k - x_{k-1}) / (x_{k+1} - x_{k-1})
 *   r = (p_d - p_c) + t ((p_u - p_c) - (p_d - p_c))        (p = y or z)
 *   chi2 = (r_y^2/sigma_y^2 + r_z^2/sigma_z^2) / (1 + t^2 + (1-t)^2)
 * The pair with the smallest (chi2, d, u) wins; it is kept if chi2 <=
 * nf_chi2_max.  Rows 0 and n_rows-1 lack a neighbour row and get no links.
 */
static double nf_pair_chi2(const sector_ctx* sc, int k, int32_t d, int32_t c, int32_t u) {
  const float* x = sc->geo->row_x;
  const double t = ((double)x[k] - (double)x[k - 1]) / ((double)x[k + 1] - (double)x[k - 1]);
  const double norm = 1.0 + t * t + (1.0 - t) * (1.0 - t);
  double yc = sc->ev->y[c], zc = sc->ev->z[c];
  double dyd = (double)sc->ev->y[d] - yc, dzd = (double)sc->ev->z[d] - zc;
  double dyu = (double)sc->ev->y[u] - yc, dzu = (double)sc->ev->z[u] - zc;
  double ry = dyd + t * (dyu - dyd);
  double rz = dzd + t * (dzu - dzd);
  double sy2 = sc->prm->sigma_y * sc->prm->sigma_y, sz2 = sc->prm->sigma_z * sc->prm->sigma_z;
  return (ry * ry / sy2 + rz * rz / sz2) / norm;
}

/* Candidates of row r inside the window of cluster c (exact criterion). */
static int64_t nf_window(const sector_ctx* sc, int r, int32_t c, int32_t* out, int64_t cap) {
  const orc_params* p = sc->prm;
  double yc = sc->ev->y[c], zc = sc->ev->z[c];
  int64_t base = sc->ro[0], end = sc->ro[r + 1] - base;
  int64_t n = 0;
  for (int64_t i = row_lower_bound(sc, r, yc - p->nf_win_y); i < end; ++i) {
    int32_t j = sc->sorted[i];
    double dy = (double)sc->ev->y[j] - yc;
    if (dy > p->nf_win_y) break;
    if (fabs(dy) <= p->nf_win_y && fabs((double)sc->ev->z[j] - zc) <= p->nf_win_z) {
      if (n < cap) out[n] = j;
      ++n;
    }
  }
  return n;
}

static void nf_row(const sector_ctx* sc, int k, int32_t* up, int32_t* dn) {
  int64_t nd_cap = sc->ro[k] - sc->ro[k - 1], nu_cap = sc->ro[k + 2] - sc->ro[k + 1];
  int32_t* D = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nd_cap + 1));
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nu_cap + 1));
  for (int32_t c = sc->ro[k]; c < sc->ro[k + 1]; ++c) {
    int64_t nd = nf_window(sc, k - 1, c, D, nd_cap);
    int64_t nu = nf_window(sc, k + 1, c, U, nu_cap);
    double best = INFINITY;
    int32_t bd = -1, bu = -1;
    for (int64_t i = 0; i < nd; ++i) {
      for (int64_t j = 0; j < nu; ++j) {
        double chi2 = nf_pair_chi2(sc, k, D[i], c, U[j]);
        int better = chi2 < best || (chi2 == best && (D[i] < bd || (D[i] == bd && U[j] < bu)));
        if (bd < 0 || better) {
          best = chi2;
          bd = D[i];
          bu = U[j];
        }
      }
    }
    if (bd >= 0 && best <= sc->prm->nf_chi2_max) {
      up[c] = bu;
      dn[c] = bd;
    } else {
      up[c] = -1;
      dn[c] = -1;
    }
  }
  free(D);
  free(U);
}

static void sector_neighbours(const sector_ctx* sc, int32_t* up, int32_t* dn) {
  int nr = sc->nr;
  for (int32_t c = sc->ro[0]; c < sc->ro[1]; ++c) up[c] = dn[c] = -1;
  if (nr >= 2)
    for (int32_t c = sc->ro[nr - 1]; c < sc->ro[nr]; ++c) up[c] = dn[c] = -1;
  for (int k = 1; k + 1 < nr; ++k) nf_row(sc, k, up, dn);
}

/* ------------------------------------------------------------------------ */
/* Evolution step (section 1, second combinatorial step)                    */
/* ------------------------------------------------------------------------ */
/* A link survives only if the neighbour links back: up'(c) = u iff dn(u) = c,
 * dn'(c) = d iff up(d) = c.  Reads the links before evolution only. */
static void evolve_range(int64_t b, int64_t e, const int32_t* up, const int32_t* dn,
                         int32_t* up2, int32_t* dn2) {
  for (int64_t c = b; c < e; ++c) {
    int32_t u = up[c], d = dn[c];
    up2[c] = (u >= 0 && dn[u] == c) ? u : -1;
    dn2[c] = (d >= 0 && up[d] == c) ? d : -1;
  }
}

int orc_evolve(int64_t n, const int32_t* up, const int32_t* dn, int32_t* up2, int32_t* dn2) {
  if (n < 0 || (n > 0 && (!up || !dn || !up2 || !dn2))) return -1;
  evolve_range(0, n, up, dn, up2, dn2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Chains of one-to-one links define the tracklets (section 1)              */
/* ------------------------------------------------------------------------ */
/* A chain starts at a cluster with an outgoing but no incoming link and is
 * followed outward.  Chains shorter than min_seed_len clusters are dropped.
 * The tracklet id is the start cluster's event-global index. */
static int chain_length(const int32_t* up2, int32_t c) {
  int m = 0;
  for (; c >= 0; c = up2[c]) ++m;
  return m;
}

static int64_t sector_seeds(const sector_ctx* sc, const int32_t* up2, const int32_t* dn2,
                            int32_t* seeds, int64_t cap) {
  int64_t n = 0;
  for (int32_t c = sc->ro[0]; c < sc->ro[sc->nr]; ++c) {
    if (dn2[c] == -1 && up2[c] != -1 && chain_length(up2, c) >= sc->prm->min_seed_len) {
      if (seeds && n < cap) seeds[n] = c;
      ++n;
    }
  }
  return n;
}

/* ------------------------------------------------------------------------ */
/* Track model: exact helix in the sector frame, Kalman filter               */
/* ------------------------------------------------------------------------ */
/*
 * The paper only says that a Kalman filter fits the tracklets.  Reading used:
 * uniform field along z, no material, state (y, z, sin phi, tan lambda, q/pT)
 * at the x of a pad row, exact propagation between rows:
 *   sin phi2 = sin phi1 - kappa dx
 *   y2 = y1 + dx (sin phi1 + sin phi2) / (cos phi1 + cos phi2)
 *   z2 = z1 + tan lambda * s, s the transverse arc length,
 *   s = dx sqrt(1+T^2) asin(u)/u, u = kappa dx sqrt(1+T^2) / 2,
 *   T = (sin phi1 + sin phi2)/(cos phi1 + cos phi2)
 * and the covariance propagated with the analytic Jacobian of that map.
 */
typedef struct {
  double x;
  double p[5];
  double C[5][5];
} kstate;

static double asinc(double u) { return u == 0.0 ? 1.0 : asin(u) / u; }

/* d/du (asin(u)/u) */
static double asinc_d(double u) {
  if (fabs(u) < 1e-4) return u / 3.0 + 0.3 * u * u * u;
  return (u / sqrt(1.0 - u * u) - asin(u)) / (u * u);
}

static void mat_jcjt(double C[5][5], double J[5][5]) {
  double T[5][5], R[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int a = 0; a < 5; ++a) s += J[i][a] * C[a][j];
      T[i][j] = s;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int a = 0; a < 5; ++a) s += T[i][a] * J[j][a];
      R[i][j] = s;
    }
  memcpy(C, R, sizeof(R));
}

/* Returns 0, or 1 when |sin phi| would pass max_sinphi (state unchanged). */
static int kprop(kstate* s, double x2, double bz, double max_sinphi, double J[5][5]) {
  const double k = CLIGHT * bz;
  const double dx = x2 - s->x;
  const double kap = k * s->p[4];
  const double s1 = s->p[2], s2 = s1 - kap * dx;
  if (fabs(s1) > max_sinphi || fabs(s2) > max_sinphi) return 1;
  const double c1 = sqrt((1.0 - s1) * (1.0 + s1)), c2 = sqrt((1.0 - s2) * (1.0 + s2));
  const double T = (s1 + s2) / (c1 + c2);
  const double Q = sqrt(1.0 + T * T);
  const double u = kap * dx * Q / 2.0;
  const double ds = dx * Q * asinc(u);
  const double tanl = s->p[3];
  /* derivatives */
  const double dT_ds1 = (1.0 + T * T) * 0.5 * (1.0 / c1 + 1.0 / c2); /* s2 moves with s1 */
  const double dT_dk = -(1.0 + T * T) * dx / (2.0 * c2);             /* at fixed s1 */
  const double dQ_ds1 = T / Q * dT_ds1, dQ_dk = T / Q * dT_dk;
  const double isq = 1.0 / sqrt(1.0 - u * u); /* d(asin u)/du */
  const double dds_ds1 = dx * dQ_ds1 * isq;
  const double dds_dk = dx * (dQ_dk * isq + Q * Q * dx * asinc_d(u) / 2.0);
  double Jl[5][5] = {{0}};
  for (int i = 0; i < 5; ++i) Jl[i][i] = 1.0;
  Jl[0][2] = dx * dT_ds1;
  Jl[0][4] = dx * dT_dk * k;
  Jl[1][2] = tanl * dds_ds1;
  Jl[1][3] = ds;
  Jl[1][4] = tanl * dds_dk * k;
  Jl[2][4] = -dx * k;
  s->p[0] += dx * T;
  s->p[1] += tanl * ds;
  s->p[2] = s2;
  s->x = x2;
  mat_jcjt(s->C, Jl);
  if (J) memcpy(J, Jl, sizeof(Jl));
  return 0;
}

/* chi^2 of measurement (my, mz) against the predicted state. */
static double kchi2(const kstate* s, double my, double mz, double sy2, double sz2) {
  double S00 = s->C[0][0] + sy2, S01 = s->C[0][1], S11 = s->C[1][1] + sz2;
  double det = S00 * S11 - S01 * S01;
  double ry = my - s->p[0], rz = mz - s->p[1];
  return (ry * ry * S11 - 2.0 * ry * rz * S01 + rz * rz * S00) / det;
}

/* Kalman update with measurement (my, mz); returns its chi^2. */
static double kupdate(kstate* s, double my, double mz, double sy2, double sz2) {
  double S00 = s->C[0][0] + sy2, S01 = s->C[0][1], S11 = s->C[1][1] + sz2;
  double det = S00 * S11 - S01 * S01;
  double i00 = S11 / det, i01 = -S01 / det, i11 = S00 / det;
  double ry = my - s->p[0], rz = mz - s->p[1];
  double chi2 = ry * ry * i00 + 2.0 * ry * rz * i01 + rz * rz * i11;
  double K[5][2], H[2][5];
  for (int j = 0; j < 5; ++j) {
    H[0][j] = s->C[0][j];
    H[1][j] = s->C[1][j];
  }
  for (int i = 0; i < 5; ++i) {
    K[i][0] = s->C[i][0] * i00 + s->C[i][1] * i01;
    K[i][1] = s->C[i][0] * i01 + s->C[i][1] * i11;
  }
  for (int i = 0; i < 5; ++i) s->p[i] += K[i][0] * ry + K[i][1] * rz;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) s->C[i][j] -= K[i][0] * H[0][j] + K[i][1] * H[1][j];
  return chi2;
}

static void kreset_cov(kstate* s, const orc_params* p) {
  memset(s->C, 0, sizeof(s->C));
  s->C[0][0] = p->sigma_y * p->sigma_y;
  s->C[1][1] = p->sigma_z * p->sigma_z;
  s->C[2][2] = p->prior_sinphi;
  s->C[3][3] = p->prior_tanl;
  s->C[4][4] = p->prior_qpt;
}

/*
 * Seed of a tracklet from three chain clusters a (first), b (middle), e
 * (last of the seed window): the circle through their (x, y) gives the
 * curvature and the direction at a; tan lambda is the z rise over the arc
 * length a -> e.
 * Positions at a are taken from cluster a.  With Bz = 0 the track is straight.
 */
static void kseed(kstate* s, double xa, double ya, double za, double xb, double yb,
                  double xe, double ye, double ze, double bz, const orc_params* p) {
  double d1x = xb - xa, d1y = yb - ya, d2x = xe - xa, d2y = ye - ya;
  double kappa = 0.0;
  if (bz != 0.0) {
    double cross = d1x * d2y - d1y * d2x;
    double den = hypot(d1x, d1y) * hypot(d2x, d2y) * hypot(d2x - d1x, d2y - d1y);
    kappa = den > 0.0 ? -2.0 * cross / den : 0.0;
  }
  double L = hypot(d2x, d2y);
  double u = kappa * L / 2.0;
  if (u > 1.0) u = 1.0;
  if (u < -1.0) u = -1.0;
  s->x = xa;
  s->p[0] = ya;
  s->p[1] = za;
  s->p[2] = (d2y / L) * sqrt(1.0 - u * u) + (d2x / L) * u;
  s->p[3] = (ze - za) / (L * asinc(u));
  s->p[4] = bz != 0.0 ? kappa / (CLIGHT * bz) : 0.0;
  kreset_cov(s, p);
}

/* ------------------------------------------------------------------------ */
/* Tracklet construction (section 1)                                         */
/* ------------------------------------------------------------------------ */
/*
 * The paper: fit the tracklet with a Kalman filter, extrapolate to adjacent
 * rows, collect clusters that meet a chi^2 condition, refit, until no more
 * clusters are found.  Reading used:
 *   1. seed from the chain (kseed: first, middle and last of the first
 *      seed_window chain clusters; the seed only starts the outward filter,
 *      and a window of 16 and the whole chain give the same tracks), then
 *      filter outward through all chain clusters unconditionally;
 *   2. keep going outward row by row: propagate, search the row, take the
 *      cluster with the smallest (chi2, index) if chi2 <= chi2_gate, else
 *      count a miss;
 *   3. refit inward from the outermost collected cluster with a fresh
 *      covariance, through all collected clusters unconditionally, and keep
 *      going inward below the innermost one with the rule of step 2.
 * A row step stops the extension when |sin phi| would exceed max_sinphi,
 * when |z| > z_max, after more than max_miss consecutive misses, or at the
 * first/last row.  A predicted y outside the sector (|y| > x tan_half) is a
 * miss.  If a step through already-collected clusters fails, the tracklet
 * is dropped (n = 0).  The chi^2 of the tracklet is the sum over the inward
 * refit (its first cluster initialises the state); ndf = 2n - 5; the output
 * state is the inward fit at the innermost collected cluster.
 */
static int32_t search_row(const sector_ctx* sc, int r, const kstate* s, double* chi2_out) {
  const orc_params* p = sc->prm;
  double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  double S00 = s->C[0][0] + sy2, S11 = s->C[1][1] + sz2;
  /* bounding box of the gate ellipse, widened slightly: only an accelerator */
  double wy = sqrt(p->chi2_gate * S00) * (1.0 + 1e-9) + 1e-12;
  double wz = sqrt(p->chi2_gate * S11) * (1.0 + 1e-9) + 1e-12;
  int64_t base = sc->ro[0], end = sc->ro[r + 1] - base;
  double best = INFINITY;
  int32_t bi = -1;
  for (int64_t i = row_lower_bound(sc, r, s->p[0] - wy); i < end; ++i) {
    int32_t j = sc->sorted[i];
    double yj = sc->ev->y[j];
    if (yj > s->p[0] + wy) break;
    double zj = sc->ev->z[j];
    if (fabs(zj - s->p[1]) > wz) continue;
    double chi2 = kchi2(s, yj, zj, sy2, sz2);
    if (chi2 <= p->chi2_gate && (chi2 < best || (chi2 == best && j < bi))) {
      best = chi2;
      bi = j;
    }
  }
  *chi2_out = best;
  return bi;
}

typedef struct {
  int32_t row_lo, row_hi, n, ndf;
  double chi2;
  double par[6];
  kstate s_in;   /* inward fit at the innermost collected cluster */
  kstate s_out;  /* outward filter at the outermost collected cluster */
} tl_result;

/* Extension step at row r: returns 0 = hit, 1 = miss, 2 = stop. */
static int extend_step(const sector_ctx* sc, kstate* s, int r, int32_t* hit, double* chi2) {
  const orc_params* p = sc->prm;
  const orc_geometry* g = sc->geo;
  double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  if (kprop(s, g->row_x[r], sc->bz, p->max_sinphi, NULL)) return 2;
  if (fabs(s->p[1]) > (double)g->z_max) return 2;
  if (fabs(s->p[0]) > (double)g->row_x[r] * (double)g->tan_half_angle) return 1;
  double c2;
  int32_t j = search_row(sc, r, s, &c2);
  if (j < 0) return 1;
  *chi2 = kupdate(s, sc->ev->y[j], sc->ev->z[j], sy2, sz2);
  *hit = j;
  return 0;
}

static void build_tracklet(const sector_ctx* sc, const int32_t* up2, int32_t start,
                           int32_t* hits, tl_result* res) {
  const orc_params* p = sc->prm;
  const float* X = sc->geo->row_x;
  const int nr = sc->nr;
  const double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  const float* Y = sc->ev->y;
  const float* Z = sc->ev->z;
  for (int r = 0; r < nr; ++r) hits[r] = -1;
  memset(res, 0, sizeof(*res));

  /* the chain */
  int32_t chain[1024];
  int m = 0;
  for (int32_t c = start; c >= 0 && m < 1024; c = up2[c]) chain[m++] = c;
  const int k0 = row_of_cluster(sc, start);
  /* the seed circle uses the first, middle and last of the first
     min(m, seed_window) chain clusters */
  int ms = m < p->seed_window ? m : p->seed_window;
  if (ms < 2) ms = m < 2 ? m : 2;
  const int32_t a = chain[0], b = chain[ms / 2], e = chain[ms - 1];

  /* 1. seed and outward filter through the chain */
  kstate s;
  kseed(&s, X[k0], Y[a], Z[a], X[k0 + ms / 2], Y[b], X[k0 + ms - 1], Y[e], Z[e], sc->bz, p);
  if (fabs(s.p[2]) > p->max_sinphi) return; /* dropped */
  hits[k0] = a;
  kstate last = s;
  int last_row = k0;
  for (int j = 1; j < m; ++j) {
    if (kprop(&s, X[k0 + j], sc->bz, p->max_sinphi, NULL)) return;
    kupdate(&s, Y[chain[j]], Z[chain[j]], sy2, sz2);
    hits[k0 + j] = chain[j];
    last = s;
    last_row = k0 + j;
  }
  /* 2. outward extension */
  int misses = 0;
  for (int r = k0 + m; r < nr; ++r) {
    int32_t h;
    double c2;
    int st = extend_step(sc, &s, r, &h, &c2);
    if (st == 2) break;
    if (st == 0) {
      hits[r] = h;
      last = s;
      last_row = r;
      misses = 0;
    } else if (++misses > p->max_miss) {
      break;
    }
  }
  /* 3. inward refit from the outermost collected cluster */
  int32_t ho = hits[last_row];
  kstate w;
  w.x = X[last_row];
  w.p[0] = Y[ho];
  w.p[1] = Z[ho];
  w.p[2] = last.p[2];
  w.p[3] = last.p[3];
  w.p[4] = last.p[4];
  kreset_cov(&w, p);
  double chi2 = 0.0;
  int n = 1, inner = last_row;
  kstate inner_s = w;
  for (int r = last_row - 1; r >= k0; --r) {
    if (kprop(&w, X[r], sc->bz, p->max_sinphi, NULL)) return; /* dropped */
    if (hits[r] >= 0) {
      chi2 += kupdate(&w, Y[hits[r]], Z[hits[r]], sy2, sz2);
      ++n;
      inner = r;
      inner_s = w;
    }
  }
  misses = 0;
  for (int r = k0 - 1; r >= 0; --r) {
    int32_t h;
    double c2 = 0.0;
    int st = extend_step(sc, &w, r, &h, &c2);
    if (st == 2) break;
    if (st == 0) {
      hits[r] = h;
      chi2 += c2;
      ++n;
      inner = r;
      inner_s = w;
      misses = 0;
    } else if (++misses > p->max_miss) {
      break;
    }
  }
  res->row_lo = inner;
  res->row_hi = last_row;
  res->n = n;
  res->ndf = 2 * n - 5;
  res->chi2 = chi2;
  res->par[0] = inner_s.x;
  for (int i = 0; i < 5; ++i) res->par[1 + i] = inner_s.p[i];
  res->s_in = inner_s;
  res->s_out = last;
}

/* ------------------------------------------------------------------------ */
/* Tracklet selection (sections 1 and 3.1)                                   */
/* ------------------------------------------------------------------------ */
/*
 * Cluster weight w = n (alpha - chi2/beta), here with the chi^2 per degree of
 * freedom of the inward fit (chi2/ndf) so that chi2/beta is of order one with
 * beta = 1.  Tracklets compete only if they pass the pre-cuts n >=
 * min_clusters and pT >= min_pt (when Bz != 0).  Each cluster goes to the
 * competing tracklet of largest weight, the smaller id winning exact ties.
 * A tracklet becomes a track if it owns >= min_clusters clusters.
 */
static int tl_qualifies(const orc_params* p, double bz, int32_t n, double qpt) {
  if (n < p->min_clusters) return 0;
  if (bz != 0.0 && fabs(qpt) > 1.0 / p->min_pt) return 0;
  return 1;
}

static double tl_weight(const orc_params* p, int32_t n, double chi2, int32_t ndf) {
  return (double)n * (p->alpha - (chi2 / (double)ndf) / p->beta);
}

/* owner_l: indexed by cluster - cbase; -1 = none.  keep: per tracklet. */
static void select_core(const orc_params* p, double bz, int32_t nr, int64_t n_tl,
                        const int32_t* ids, const int32_t* hits, const int32_t* row_lo,
                        const int32_t* row_hi, const int32_t* n, const double* chi2,
                        const int32_t* ndf, const double* par, const double* weights,
                        int64_t cbase, int64_t ncl, int32_t* owner_l, int32_t* keep) {
  double* wbest = (double*)malloc(sizeof(double) * (size_t)(ncl > 0 ? ncl : 1));
  for (int64_t c = 0; c < ncl; ++c) owner_l[c] = -1;
  for (int64_t t = 0; t < n_tl; ++t) {
    keep[t] = 0;
    if (!tl_qualifies(p, bz, n[t], par[6 * t + 5])) continue;
    double w = weights ? weights[t] : tl_weight(p, n[t], chi2[t], ndf[t]);
    for (int r = row_lo[t]; r <= row_hi[t]; ++r) {
      int32_t c = hits[t * nr + r];
      if (c < 0) continue;
      int64_t lc = c - cbase;
      int32_t o = owner_l[lc];
      if (o < 0 || w > wbest[lc] || (w == wbest[lc] && ids[t] < ids[o])) {
        owner_l[lc] = (int32_t)t;
        wbest[lc] = w;
      }
    }
  }
  for (int64_t t = 0; t < n_tl; ++t) {
    if (n[t] <= 0) continue;
    int32_t owned = 0;
    for (int r = row_lo[t]; r <= row_hi[t]; ++r) {
      int32_t c = hits[t * nr + r];
      if (c >= 0 && owner_l[c - cbase] == t) ++owned;
    }
    keep[t] = owned >= p->min_clusters;
  }
  free(wbest);
}

/* ------------------------------------------------------------------------ */
/* Per-sector driver                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n_tracks, n_clusters;
  double* par;       /* [n_tracks][8] */
  int32_t* meta;     /* [n_tracks][4] (first relative to this sector) */
  int32_t* clusters; /* [n_clusters] */
  kstate* ends;      /* [n_tracks][2]: inner and outer end states */
  int32_t* end_rows; /* [n_tracks][2]: their rows */
  int status;
} sector_out;

static void track_sector(const orc_event* ev, const orc_geometry* geo, double bz,
                         const orc_params* prm, int slot, int32_t* up, int32_t* dn,
                         int32_t* up2, int32_t* dn2, sector_out* so) {
  memset(so, 0, sizeof(*so));
  sector_ctx sc;
  if (sector_init(&sc, ev, geo, prm, bz, slot)) {
    so->status = -1;
    return;
  }
  const int nr = sc.nr;
  const int64_t cbase = sc.ro[0], ncl = sc.ro[nr] - cbase;
  sector_neighbours(&sc, up, dn);
  evolve_range(cbase, cbase + ncl, up, dn, up2, dn2);
  int64_t n_tl = sector_seeds(&sc, up2, dn2, NULL, 0);
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tl + 1));
  sector_seeds(&sc, up2, dn2, ids, n_tl);
  int32_t* hits = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tl * nr + 1));
  int32_t* row_lo = (int32_t*)calloc((size_t)(n_tl + 1), sizeof(int32_t));
  int32_t* row_hi = (int32_t*)calloc((size_t)(n_tl + 1), sizeof(int32_t));
  int32_t* nn = (int32_t*)calloc((size_t)(n_tl + 1), sizeof(int32_t));
  int32_t* ndf = (int32_t*)calloc((size_t)(n_tl + 1), sizeof(int32_t));
  double* chi2 = (double*)calloc((size_t)(n_tl + 1), sizeof(double));
  double* par = (double*)calloc((size_t)(6 * n_tl + 1), sizeof(double));
  kstate* ends = (kstate*)malloc(sizeof(kstate) * (size_t)(2 * n_tl + 1));
  for (int64_t t = 0; t < n_tl; ++t) {
    tl_result res;
    build_tracklet(&sc, up2, ids[t], hits + t * nr, &res);
    ends[2 * t] = res.s_in;
    ends[2 * t + 1] = res.s_out;
    row_lo[t] = res.row_lo;
    row_hi[t] = res.row_hi;
    nn[t] = res.n;
    ndf[t] = res.ndf;
    chi2[t] = res.chi2;
    memcpy(par + 6 * t, res.par, sizeof(res.par));
  }
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncl + 1));
  int32_t* keep = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tl + 1));
  select_core(prm, bz, nr, n_tl, ids, hits, row_lo, row_hi, nn, chi2, ndf, par, NULL, cbase, ncl,
              owner, keep);
  /* output: kept tracklets in id order, owned clusters in row order */
  int64_t nt = 0, nc = 0;
  for (int64_t t = 0; t < n_tl; ++t) {
    if (!keep[t]) continue;
    ++nt;
    for (int r = row_lo[t]; r <= row_hi[t]; ++r) {
      int32_t c = hits[t * nr + r];
      if (c >= 0 && owner[c - cbase] == t) ++nc;
    }
  }
  so->n_tracks = nt;
  so->n_clusters = nc;
  so->par = (double*)malloc(sizeof(double) * (size_t)(8 * nt + 1));
  so->meta = (int32_t*)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
  so->clusters = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc + 1));
  so->ends = (kstate*)malloc(sizeof(kstate) * (size_t)(2 * nt + 1));
  so->end_rows = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * nt + 1));
  int64_t it = 0, ic = 0;
  for (int64_t t = 0; t < n_tl; ++t) {
    if (!keep[t]) continue;
    int64_t first = ic;
    for (int r = row_lo[t]; r <= row_hi[t]; ++r) {
      int32_t c = hits[t * nr + r];
      if (c >= 0 && owner[c - cbase] == t) so->clusters[ic++] = c;
    }
    for (int i = 0; i < 6; ++i) so->par[8 * it + i] = par[6 * t + i];
    so->par[8 * it + 6] = chi2[t];
    so->par[8 * it + 7] = ndf[t];
    so->meta[4 * it + 0] = ev->sector_id[slot];
    so->meta[4 * it + 1] = (int32_t)(ic - first);
    so->meta[4 * it + 2] = (int32_t)first;
    so->meta[4 * it + 3] = ids[t];
    so->ends[2 * it] = ends[2 * t];
    so->ends[2 * it + 1] = ends[2 * t + 1];
    so->end_rows[2 * it] = row_lo[t];
    so->end_rows[2 * it + 1] = row_hi[t];
    ++it;
  }
  free(ids); free(hits); free(row_lo); free(row_hi); free(nn); free(ndf); free(chi2);
  free(par); free(owner); free(keep); free(ends);
  sector_free(&sc);
}

typedef struct {
  const orc_event* ev;
  const orc_geometry* geo;
  const orc_params* prm;
  double bz;
  int32_t *up, *dn, *up2, *dn2;
  sector_out* outs;
  int next;
  pthread_mutex_t lock;
} pool_t;

static void* pool_worker(void* arg) {
  pool_t* P = (pool_t*)arg;
  for (;;) {
    pthread_mutex_lock(&P->lock);
    int slot = P->next++;
    pthread_mutex_unlock(&P->lock);
    if (slot >= P->ev->n_sectors) break;
    track_sector(P->ev, P->geo, P->bz, P->prm, slot, P->up, P->dn, P->up2, P->dn2,
                 &P->outs[slot]);
  }
  return NULL;
}

static int check_event(const orc_event* ev, const orc_geometry* geo) {
  if (!ev || !geo || !geo->row_x || geo->n_rows < 3 || geo->n_rows > 1024) return -1;
  if (ev->n_sectors < 0) return -1;
  if (ev->n_clusters > 0 && (!ev->y || !ev->z)) return -1;
  if (!ev->row_offsets || !ev->sector_id) return -1;
  int64_t nrs = (int64_t)ev->n_sectors * geo->n_rows;
  if (ev->row_offsets[0] != 0 || ev->row_offsets[nrs] != ev->n_clusters) return -1;
  for (int64_t i = 0; i < nrs; ++i)
    if (ev->row_offsets[i + 1] < ev->row_offsets[i]) return -1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Global tracking (section 5)                                               */
/* ------------------------------------------------------------------------ */
/*
 * A sector track needs min_clusters clusters, so the part of a track beyond a
 * sector boundary that is too short to be a sector track of its own is not
 * found.  The paper prolongs the track segments that end at a sector edge:
 * their parameters are converted to the neighbouring sector's frame and the
 * tracklet construction continues there.  Reading used:
 *   - both ends of every sector track are tried: the inner end starts from
 *     the inward fit at the innermost cluster, the outer end from the
 *     outward filter at the outermost cluster (state and covariance);
 *   - from the end, the track is propagated row by row away from its
 *     clusters (inward: decreasing rows) in its own sector, without search
 *     (those rows were searched by the sector tracker); if at some row it is
 *     outside the trapezoid (|y| > x tan_half) it has left through the side
 *     edge; reaching the first/last row, |sin phi| > max_sinphi or
 *     |z| > z_max ends it without prolongation;
 *   - the neighbour is the sector on that side: same z half (section 1:
 *     2 x 18 sectors, ids 0-17 and 18-35), sector index +1 (mod 18) for
 *     y > 0, -1 for y < 0, if the event holds it (its first slot with that
 *     id); a slot whose id is outside 0-35 is not prolonged; its centre line is one sector width (2 atan of
 *     tan_half) away;
 *   - the state at the last row inside the own sector is rotated into the
 *     neighbour's frame (krotate), so that the neighbour's rows crossed
 *     between the edge and the next own row are not skipped, and the
 *     construction continues from the first row beyond the rotated x in the
 *     same direction (rows where the track is outside the neighbour's
 *     trapezoid hold none of its clusters and count as misses), with the sector tracker's extension rule (chi^2 gate,
 *     stop after more than max_miss consecutive misses, same stops), taking
 *     only clusters that no sector track owns;
 *   - a free cluster taken by several prolongations goes to the one with the
 *     smallest (seed id of its track, end); each prolongation keeps the
 *     clusters it owns (at least one, else it is not reported) and reports
 *     the state of its own fit at its last collected cluster, the chi^2 of
 *     its updates and ndf = 2 per collected cluster.
 */

/* Rotation of the local frame by d (radians; the new x axis at angle d from
 * the old one).  The point and the direction stay; the reference x becomes
 * the rotated x.  For the covariance, a change of the old y at fixed old x
 * is brought back onto the new reference plane along the track: the
 * Jacobian has dy'/dy = cos(phi)/cos(phi'), dz'/dy = -sin(d) tan(lambda) /
 * cos(phi'), d sin(phi')/dy = kappa sin(d) (the turn over that path) and
 * d sin(phi')/d sin(phi) = cos(phi')/cos(phi).  Returns 1, state unchanged,
 * if the direction would not point along +x' (cos(phi') <= 0). */
static int krotate(kstate* s, double d, double bz) {
  const double ca = cos(d), sa = sin(d);
  const double sp = s->p[2], cp = sqrt((1.0 - sp) * (1.0 + sp));
  const double sp2 = sp * ca - cp * sa, cp2 = cp * ca + sp * sa;
  if (!(cp2 > 0.0)) return 1;
  double J[5][5] = {{0}};
  J[0][0] = cp / cp2;
  J[1][0] = -sa * s->p[3] / cp2;
  J[1][1] = 1.0;
  J[2][0] = CLIGHT * bz * s->p[4] * sa;
  J[2][2] = cp2 / cp;
  J[3][3] = 1.0;
  J[4][4] = 1.0;
  const double x2 = s->x * ca + s->p[0] * sa, y2 = -s->x * sa + s->p[0] * ca;
  s->x = x2;
  s->p[0] = y2;
  s->p[2] = sp2;
  mat_jcjt(s->C, J);
  return 0;
}

/* search_row among the clusters no track owns (cluster_track < 0). */
static int32_t search_row_free(const sector_ctx* sc, int r, const kstate* s,
                               const int32_t* cluster_track) {
  const orc_params* p = sc->prm;
  double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  double S00 = s->C[0][0] + sy2, S11 = s->C[1][1] + sz2;
  double wy = sqrt(p->chi2_gate * S00) * (1.0 + 1e-9) + 1e-12;
  double wz = sqrt(p->chi2_gate * S11) * (1.0 + 1e-9) + 1e-12;
  int64_t base = sc->ro[0], end = sc->ro[r + 1] - base;
  double best = INFINITY;
  int32_t bi = -1;
  for (int64_t i = row_lower_bound(sc, r, s->p[0] - wy); i < end; ++i) {
    int32_t j = sc->sorted[i];
    double yj = sc->ev->y[j];
    if (yj > s->p[0] + wy) break;
    if (cluster_track[j] >= 0) continue;
    double zj = sc->ev->z[j];
    if (fabs(zj - s->p[1]) > wz) continue;
    double chi2 = kchi2(s, yj, zj, sy2, sz2);
    if (chi2 <= p->chi2_gate && (chi2 < best || (chi2 == best && j < bi))) {
      best = chi2;
      bi = j;
    }
  }
  return bi;
}

typedef struct {
  int32_t track, end, seed, sector_id, n;
  int32_t* cl;   /* [n_rows] collected clusters in the order met */
  double chi2;
  kstate fin;
} prol_t;

/* Prolongation of one end of one track; returns 1 if it collected clusters. */
static int prolong_one(const orc_event* ev, const orc_geometry* geo, double bz,
                       const orc_params* p, const sector_ctx* ctx, const int* phys2slot,
                       int slot, const kstate* start, int row, int dir,
                       const int32_t* cluster_track, prol_t* out) {
  const int nr = geo->n_rows;
  const double th = (double)geo->tan_half_angle;
  const double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  kstate s = *start, last = *start;
  /* 1. own sector: propagate until the track leaves through a side edge;
   * `last` is the state at the last row inside */
  int exit_row = -1;
  for (int r = row + dir; r >= 0 && r < nr; r += dir) {
    if (kprop(&s, geo->row_x[r], bz, p->max_sinphi, NULL)) return 0;
    if (fabs(s.p[1]) > (double)geo->z_max) return 0;
    if (fabs(s.p[0]) > (double)geo->row_x[r] * th) {
      exit_row = r;
      break;
    }
    last = s;
  }
  if (exit_row < 0) return 0;
  /* 2. the neighbour on that side */
  const int phys = ev->sector_id[slot];
  if (phys < 0 || phys >= 36) return 0;  /* not a sector of the 2 x 18 layout */
  const int half = phys / 18, idx = phys % 18;
  const int up = s.p[0] > 0.0;
  s = last;
  const int nphys = half * 18 + (idx + (up ? 1 : 17)) % 18;
  const int nslot = (nphys >= 0 && nphys < 36) ? phys2slot[nphys] : -1;
  if (nslot < 0) return 0;
  /* neighbouring sectors' centre lines are one sector width apart */
  const double width = 2.0 * atan(th);
  if (krotate(&s, (up ? 1.0 : -1.0) * width, bz)) return 0;
  if (fabs(s.p[2]) > p->max_sinphi) return 0;
  /* 3. continue the construction there, from the first row beyond x */
  int r = dir < 0 ? nr - 1 : 0;
  if (dir < 0)
    while (r >= 0 && (double)geo->row_x[r] >= s.x) --r;
  else
    while (r < nr && (double)geo->row_x[r] <= s.x) ++r;
  const sector_ctx* sc = &ctx[nslot];
  int misses = 0, n = 0;
  double chi2 = 0.0;
  for (; r >= 0 && r < nr; r += dir) {
    if (kprop(&s, geo->row_x[r], bz, p->max_sinphi, NULL)) break;
    if (fabs(s.p[1]) > (double)geo->z_max) break;
    int32_t h = -1;
    if (!(fabs(s.p[0]) > (double)geo->row_x[r] * th)) h = search_row_free(sc, r, &s, cluster_track);
    if (h >= 0) {
      chi2 += kupdate(&s, sc->ev->y[h], sc->ev->z[h], sy2, sz2);
      out->cl[n++] = h;
      out->fin = s;
      misses = 0;
    } else if (++misses > p->max_miss) {
      break;
    }
  }
  if (n == 0) return 0;
  out->n = n;
  out->chi2 = chi2;
  out->sector_id = nphys;
  return 1;
}

static int global_tracking(const orc_event* ev, const orc_geometry* geo, double bz,
                           const orc_params* prm, const sector_out* outs,
                           const orc_tracks* trk, orc_prolongations* pro) {
  const int nr = geo->n_rows;
  int phys2slot[36];
  for (int i = 0; i < 36; ++i) phys2slot[i] = -1;
  for (int sl = 0; sl < ev->n_sectors; ++sl) {
    int ph = ev->sector_id[sl];
    if (ph >= 0 && ph < 36 && phys2slot[ph] < 0) phys2slot[ph] = sl;
  }
  sector_ctx* ctx = (sector_ctx*)calloc((size_t)(ev->n_sectors + 1), sizeof(sector_ctx));
  for (int sl = 0; sl < ev->n_sectors; ++sl)
    if (sector_init(&ctx[sl], ev, geo, prm, bz, sl)) {
      for (int k = 0; k < sl; ++k) sector_free(&ctx[k]);
      free(ctx);
      return -1;
    }
  int64_t nt = trk->n_tracks;
  prol_t* pr = (prol_t*)calloc((size_t)(2 * nt + 1), sizeof(prol_t));
  int32_t* pool = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * nt * nr + 1));
  int64_t np = 0, it = 0;
  for (int sl = 0; sl < ev->n_sectors; ++sl) {
    const sector_out* so = &outs[sl];
    for (int64_t t = 0; t < so->n_tracks; ++t, ++it)
      for (int end = 0; end < 2; ++end) {
        prol_t* q = &pr[np];
        q->cl = pool + np * nr;
        q->track = (int32_t)it;
        q->end = end;
        q->seed = so->meta[4 * t + 3];
        if (prolong_one(ev, geo, bz, prm, ctx, phys2slot, sl, &so->ends[2 * t + end],
                        so->end_rows[2 * t + end], end ? 1 : -1, trk->cluster_track, q))
          ++np;
      }
  }
  /* free clusters claimed several times: smallest (seed id, end) wins */
  int64_t N = ev->n_clusters;
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  for (int64_t c = 0; c < N; ++c) owner[c] = -1;
  for (int64_t k = 0; k < np; ++k)
    for (int32_t j = 0; j < pr[k].n; ++j) {
      int32_t c = pr[k].cl[j];
      int32_t o = owner[c];
      if (o < 0 || pr[k].seed < pr[o].seed || (pr[k].seed == pr[o].seed && pr[k].end < pr[o].end))
        owner[c] = (int32_t)k;
    }
  int64_t n_out = 0, n_cl = 0;
  for (int64_t k = 0; k < np; ++k) {
    int32_t own = 0;
    for (int32_t j = 0; j < pr[k].n; ++j) own += owner[pr[k].cl[j]] == k;
    if (own > 0) {
      ++n_out;
      n_cl += own;
    }
  }
  pro->n = (int32_t)n_out;
  pro->n_clusters = (int32_t)n_cl;
  int status = (n_out > pro->cap || n_cl > pro->cap_clusters) ? 1 : 0;
  if (status == 0) {
    int64_t io = 0, ic = 0;
    for (int64_t k = 0; k < np; ++k) {  /* already in (track, end) order */
      int64_t first = ic;
      for (int32_t j = 0; j < pr[k].n; ++j)
        if (owner[pr[k].cl[j]] == k) pro->cluster[ic++] = pr[k].cl[j];
      if (ic == first) continue;
      double* P = pro->par + 8 * io;
      P[0] = pr[k].fin.x;
      for (int i = 0; i < 5; ++i) P[1 + i] = pr[k].fin.p[i];
      P[6] = pr[k].chi2;
      P[7] = 2.0 * pr[k].n;
      int32_t* M = pro->meta + 5 * io;
      M[0] = pr[k].track;
      M[1] = pr[k].end;
      M[2] = pr[k].sector_id;
      M[3] = (int32_t)(ic - first);
      M[4] = (int32_t)first;
      ++io;
    }
  }
  free(owner); free(pool); free(pr);
  for (int sl = 0; sl < ev->n_sectors; ++sl) sector_free(&ctx[sl]);
  free(ctx);
  return status;
}

static int locate(const orc_event* ev, const orc_geometry* geo, int32_t c, int* row);
static int merge_tracks(const orc_event* ev, const orc_geometry* geo, double bz,
                        const orc_params* prm, double cut, const sector_out* outs,
                        const orc_tracks* trk, const orc_prolongations* pro, orc_merged* mrg);

static int track_all(const orc_event* ev, const orc_geometry* geo, double bz,
                     const orc_params* prm, orc_tracks* out, orc_prolongations* pro,
                     orc_merged* mrg, double merge_chi2, int n_threads) {
  if (check_event(ev, geo) || !prm || !out) return -1;
  int64_t N = ev->n_clusters;
  size_t nb = sizeof(int32_t) * (size_t)(N > 0 ? N : 1);
  pool_t P;
  P.ev = ev; P.geo = geo; P.prm = prm; P.bz = bz;
  P.up = (int32_t*)malloc(nb); P.dn = (int32_t*)malloc(nb);
  P.up2 = (int32_t*)malloc(nb); P.dn2 = (int32_t*)malloc(nb);
  P.outs = (sector_out*)calloc((size_t)(ev->n_sectors + 1), sizeof(sector_out));
  P.next = 0;
  pthread_mutex_init(&P.lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > ev->n_sectors) n_threads = ev->n_sectors > 0 ? ev->n_sectors : 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, pool_worker, &P);
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&P.lock);
  int64_t nt = 0, nc = 0;
  int status = 0;
  for (int s = 0; s < ev->n_sectors; ++s) {
    nt += P.outs[s].n_tracks;
    nc += P.outs[s].n_clusters;
    if (P.outs[s].status) status = -1;
  }
  out->n_tracks = (int32_t)nt;
  out->n_track_clusters = (int32_t)nc;
  if (status == 0 && (nt > out->cap_tracks || nc > out->cap_track_clusters)) status = 1;
  if (status == 0) {
    for (int64_t c = 0; c < N; ++c) out->cluster_track[c] = -1;
    int64_t it = 0, ic = 0;
    for (int s = 0; s < ev->n_sectors; ++s) {
      sector_out* so = &P.outs[s];
      for (int64_t t = 0; t < so->n_tracks; ++t, ++it) {
        memcpy(out->track_par + 8 * it, so->par + 8 * t, 8 * sizeof(double));
        out->track_meta[4 * it + 0] = so->meta[4 * t + 0];
        out->track_meta[4 * it + 1] = so->meta[4 * t + 1];
        out->track_meta[4 * it + 2] = (int32_t)(so->meta[4 * t + 2] + ic);
        out->track_meta[4 * it + 3] = so->meta[4 * t + 3];
        for (int32_t j = 0; j < so->meta[4 * t + 1]; ++j)
          out->cluster_track[so->clusters[so->meta[4 * t + 2] + j]] = (int32_t)it;
      }
      memcpy(out->track_cluster + ic, so->clusters, sizeof(int32_t) * (size_t)so->n_clusters);
      ic += so->n_clusters;
    }
    if (pro) status = global_tracking(ev, geo, bz, prm, P.outs, out, pro);
    if (mrg && status == 0)
      status = merge_tracks(ev, geo, bz, prm, merge_chi2, P.outs, out, pro, mrg);
  }
  for (int s = 0; s < ev->n_sectors; ++s) {
    free(P.outs[s].par); free(P.outs[s].meta); free(P.outs[s].clusters);
    free(P.outs[s].ends); free(P.outs[s].end_rows);
  }
  free(P.outs); free(P.up); free(P.dn); free(P.up2); free(P.dn2);
  return status;
}

int orc_track_event(const orc_event* ev, const orc_geometry* geo, double bz,
                    const orc_params* prm, orc_tracks* out, int n_threads) {
  return track_all(ev, geo, bz, prm, out, NULL, NULL, 0.0, n_threads);
}

int orc_track_event_global(const orc_event* ev, const orc_geometry* geo, double bz,
                           const orc_params* prm, orc_tracks* out, orc_prolongations* pro,
                           int n_threads) {
  if (!pro) return -1;
  return track_all(ev, geo, bz, prm, out, pro, NULL, 0.0, n_threads);
}

int orc_track_event_merged(const orc_event* ev, const orc_geometry* geo, double bz,
                           const orc_params* prm, double merge_chi2, orc_tracks* out,
                           orc_prolongations* pro, orc_merged* mrg, int n_threads) {
  if (!mrg || !mrg->track_merged || !(merge_chi2 >= 0.0)) return -1;
  return track_all(ev, geo, bz, prm, out, pro, mrg, merge_chi2, n_threads);
}

int orc_rotate(double x, const double* st, const double* cov, double d, double bz,
               double* x_out, double* st_out, double* cov_out) {
  if (!st || !x_out || !st_out) return -1;
  kstate s;
  s.x = x;
  for (int i = 0; i < 5; ++i) s.p[i] = st[i];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) s.C[i][j] = cov ? cov[5 * i + j] : 0.0;
  if (krotate(&s, d, bz)) return 1;
  *x_out = s.x;
  for (int i = 0; i < 5; ++i) st_out[i] = s.p[i];
  if (cov_out)
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) cov_out[5 * i + j] = s.C[i][j];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Track merger with refit                                                   */
/* ------------------------------------------------------------------------ */
/*
 * After the sector tracker, the track merger joins the sector tracks of one
 * particle and refits each joined track from its cluster list alone, so
 * that the same clusters always give the same fit whatever the sector
 * tracker computed on the way (section 3.3).  The paper gives no more
 * detail; reading used:
 *   - a join links the outer end of a track A to the inner end of a track B
 *     in a side neighbour of A's sector (same half, index +-1 mod 18) or in
 *     its membrane partner (same index, other half), if B's innermost
 *     cluster is farther from the beam axis than A's outermost (joins go
 *     outward; tracks that curl back are not joined): A's outward filter at
 *     its outermost cluster is rotated into B's frame and propagated to the x
 *     of B's inward fit at its innermost cluster; the two estimates are
 *     independent, so chi^2 = d^T (C_A + C_B)^-1 d over the five parameters
 *     follows chi^2(5) for the same particle; candidates need chi^2 <=
 *     merge_chi2;
 *   - A and B are linked if each is the other's best candidate (smallest
 *     chi^2, then smallest track index); links form chains; a chain that
 *     closes on itself starts at its smallest track index;
 *   - a joined track's cluster list, in path order: the inner prolongation
 *     of its first track (outward order), each track's own clusters (row
 *     order), the outer prolongation of its last track; prolongations at the
 *     joins are not used;
 *   - refit (refit_list): the seed circle of the first run of at least three
 *     consecutive clusters of one sector with increasing rows (its first
 *     min(m, seed_window) clusters, as for a tracklet), an outward filter
 *     from there to the end of the list, then an inward fit from the last
 *     cluster with a fresh covariance over the whole list; between clusters
 *     of different sectors the state is rotated into the next sector's frame
 *     (a multiple of the sector width); a cluster whose step fails
 *     (|sin phi| limit, rotation) is skipped; the result is the inward fit at
 *     the innermost fitted cluster, with its chi^2 and ndf = 2n - 5; fewer
 *     than three fitted clusters, or a list over several sectors with an id
 *     outside 0-35, fail (ndf 0).
 */

static int frame_steps(int p, int q) {
  int k = (q % 18) - (p % 18);
  if (k > 8) k -= 18;
  if (k < -9) k += 18;
  return k;
}

typedef struct {
  double par[8];
  int32_t frame;   /* sector_id of the frame of par, -1 if failed */
  int32_t n;
} refit_res;

static int refit_list(const orc_event* ev, const orc_geometry* geo, double bz,
                      const orc_params* p, int32_t n, const int32_t* cl, refit_res* out) {
  memset(out, 0, sizeof(*out));
  out->frame = -1;
  if (n < 3) return 1;
  const float* X = geo->row_x;
  const float* Y = ev->y;
  const float* Z = ev->z;
  const double width = 2.0 * atan((double)geo->tan_half_angle);
  const double sy2 = p->sigma_y * p->sigma_y, sz2 = p->sigma_z * p->sigma_z;
  int* slot = (int*)malloc(sizeof(int) * (size_t)n);
  int* row = (int*)malloc(sizeof(int) * (size_t)n);
  int status = 1, multi = 0;
  for (int32_t j = 0; j < n; ++j) {
    slot[j] = locate(ev, geo, cl[j], &row[j]);
    if (slot[j] < 0) goto done;
    multi |= slot[j] != slot[0];
  }
  if (multi)
    for (int32_t j = 0; j < n; ++j) {
      int ph = ev->sector_id[slot[j]];
      if (ph < 0 || ph >= 36) goto done;
    }
  /* seed: first run of >= 3 same-sector clusters with increasing rows */
  int32_t i0 = -1;
  for (int32_t i = 0; i + 2 < n; ++i)
    if (slot[i + 1] == slot[i] && slot[i + 2] == slot[i] && row[i] < row[i + 1] &&
        row[i + 1] < row[i + 2]) {
      i0 = i;
      break;
    }
  if (i0 < 0) goto done;
  int32_t m = 1;
  while (i0 + m < n && m < p->seed_window && slot[i0 + m] == slot[i0] &&
         row[i0 + m] > row[i0 + m - 1])
    ++m;
  {
    const int32_t a = i0, b = i0 + m / 2, e = i0 + m - 1;
    kstate s;
    kseed(&s, X[row[a]], Y[cl[a]], Z[cl[a]], X[row[b]], Y[cl[b]], X[row[e]], Y[cl[e]], Z[cl[e]],
          bz, p);
    if (fabs(s.p[2]) > p->max_sinphi) goto done;
    /* outward filter */
    int fr = slot[i0];
    int32_t last = i0;
    for (int32_t j = i0 + 1; j < n; ++j) {
      kstate t = s;
      if (slot[j] != fr &&
          krotate(&t, frame_steps(ev->sector_id[fr], ev->sector_id[slot[j]]) * width, bz))
        continue;
      if (kprop(&t, X[row[j]], bz, p->max_sinphi, NULL)) continue;
      kupdate(&t, Y[cl[j]], Z[cl[j]], sy2, sz2);
      s = t;
      fr = slot[j];
      last = j;
    }
    /* inward fit from the last cluster, fresh covariance */
    kstate w;
    w.x = X[row[last]];
    w.p[0] = Y[cl[last]];
    w.p[1] = Z[cl[last]];
    w.p[2] = s.p[2];
    w.p[3] = s.p[3];
    w.p[4] = s.p[4];
    kreset_cov(&w, p);
    double chi2 = 0.0;
    int32_t nn = 1;
    kstate inner = w;
    int ifr = slot[last];
    for (int32_t j = last - 1; j >= 0; --j) {
      kstate t = w;
      if (slot[j] != fr &&
          krotate(&t, frame_steps(ev->sector_id[fr], ev->sector_id[slot[j]]) * width, bz))
        continue;
      if (kprop(&t, X[row[j]], bz, p->max_sinphi, NULL)) continue;
      chi2 += kupdate(&t, Y[cl[j]], Z[cl[j]], sy2, sz2);
      w = t;
      fr = slot[j];
      ++nn;
      inner = w;
      ifr = fr;
    }
    if (nn < 3) goto done;
    out->par[0] = inner.x;
    for (int i = 0; i < 5; ++i) out->par[1 + i] = inner.p[i];
    out->par[6] = chi2;
    out->par[7] = 2.0 * nn - 5.0;
    out->frame = ev->sector_id[ifr];
    out->n = nn;
    status = 0;
  }
done:
  free(slot);
  free(row);
  return status;
}

/* chi^2 of joining A's outer end to B's inner end, or -1 if they cannot join */
static double join_chi2(const kstate* a_out, int pa, const kstate* b_in, int pb, double bz,
                        const orc_params* p, double width, double cut) {
  /* tan(lambda) and q/pT are unchanged by rotation and propagation, and so
   * are their variances: d_i^2 / S_ii <= chi^2 for any positive-definite S,
   * so these two bounds reject exactly */
  for (int i = 3; i < 5; ++i) {
    double d = b_in->p[i] - a_out->p[i], v = a_out->C[i][i] + b_in->C[i][i];
    if (d * d > cut * v) return -1.0;
  }
  /* outward only: B starts farther from the beam than A ends (the radius
   * does not depend on the frame); otherwise A's outer end, propagated
   * backwards, would also match the inner end of the track it continues */
  if (!(hypot(b_in->x, b_in->p[0]) > hypot(a_out->x, a_out->p[0]))) return -1.0;
  kstate t = *a_out;
  int k = frame_steps(pa, pb);
  if (k != 0 && krotate(&t, k * width, bz)) return -1.0;
  if (kprop(&t, b_in->x, bz, p->max_sinphi, NULL)) return -1.0;
  double S[5][5], d[5];
  for (int i = 0; i < 5; ++i) {
    d[i] = b_in->p[i] - t.p[i];
    for (int j = 0; j < 5; ++j) S[i][j] = t.C[i][j] + b_in->C[i][j];
  }
  /* Cholesky S = L L^T, then chi^2 = |L^-1 d|^2 */
  double L[5][5] = {{0}};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = S[i][j];
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      if (i == j) {
        if (!(v > 0.0)) return -1.0;
        L[i][i] = sqrt(v);
      } else {
        L[i][j] = v / L[j][j];
      }
    }
  double chi2 = 0.0, yv[5];
  for (int i = 0; i < 5; ++i) {
    double v = d[i];
    for (int q = 0; q < i; ++q) v -= L[i][q] * yv[q];
    yv[i] = v / L[i][i];
    chi2 += yv[i] * yv[i];
  }
  return chi2;
}

static int merge_tracks(const orc_event* ev, const orc_geometry* geo, double bz,
                        const orc_params* prm, double cut, const sector_out* outs,
                        const orc_tracks* trk, const orc_prolongations* pro, orc_merged* mrg) {
  const int64_t nt = trk->n_tracks;
  const double width = 2.0 * atan((double)geo->tan_half_angle);
  int phys2slot[36];
  for (int i = 0; i < 36; ++i) phys2slot[i] = -1;
  for (int sl = 0; sl < ev->n_sectors; ++sl) {
    int ph = ev->sector_id[sl];
    if (ph >= 0 && ph < 36 && phys2slot[ph] < 0) phys2slot[ph] = sl;
  }
  size_t nb = (size_t)(nt + 1);
  int32_t* slot_of = (int32_t*)malloc(sizeof(int32_t) * nb);
  const kstate** e_in = (const kstate**)malloc(sizeof(kstate*) * nb);
  const kstate** e_out = (const kstate**)malloc(sizeof(kstate*) * nb);
  int64_t* first_of_slot = (int64_t*)calloc((size_t)ev->n_sectors + 1, sizeof(int64_t));
  {
    int64_t it = 0;
    for (int sl = 0; sl < ev->n_sectors; ++sl) {
      first_of_slot[sl] = it;
      for (int64_t t = 0; t < outs[sl].n_tracks; ++t, ++it) {
        slot_of[it] = sl;
        e_in[it] = &outs[sl].ends[2 * t];
        e_out[it] = &outs[sl].ends[2 * t + 1];
      }
    }
    first_of_slot[ev->n_sectors] = it;
  }
  int32_t* best_next = (int32_t*)malloc(sizeof(int32_t) * nb);
  int32_t* best_prev = (int32_t*)malloc(sizeof(int32_t) * nb);
  double* chi_next = (double*)malloc(sizeof(double) * nb);
  double* chi_prev = (double*)malloc(sizeof(double) * nb);
  for (int64_t i = 0; i < nt; ++i) {
    best_next[i] = best_prev[i] = -1;
    chi_next[i] = chi_prev[i] = INFINITY;
  }
  for (int64_t a = 0; a < nt; ++a) {
    const int pa = ev->sector_id[slot_of[a]];
    if (pa < 0 || pa >= 36) continue;
    const int half = pa / 18, idx = pa % 18;
    int cand[3] = {phys2slot[half * 18 + (idx + 1) % 18], phys2slot[half * 18 + (idx + 17) % 18],
                   phys2slot[(pa + 18) % 36]};
    for (int c = 0; c < 3; ++c) {
      const int sb = cand[c];
      if (sb < 0 || sb == slot_of[a]) continue;
      int dup = 0;
      for (int c2 = 0; c2 < c; ++c2) dup |= cand[c2] == sb;
      if (dup) continue;
      const int pb = ev->sector_id[sb];
      for (int64_t b = first_of_slot[sb]; b < first_of_slot[sb + 1]; ++b) {
        double x2 = join_chi2(e_out[a], pa, e_in[b], pb, bz, prm, width, cut);
        if (x2 < 0.0 || x2 > cut) continue;
        if (x2 < chi_next[a] || (x2 == chi_next[a] && b < best_next[a])) {
          chi_next[a] = x2;
          best_next[a] = (int32_t)b;
        }
        if (x2 < chi_prev[b] || (x2 == chi_prev[b] && a < best_prev[b])) {
          chi_prev[b] = x2;
          best_prev[b] = (int32_t)a;
        }
      }
    }
  }
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * nb);
  int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * nb);
  for (int64_t i = 0; i < nt; ++i) next[i] = prev[i] = -1;
  for (int64_t a = 0; a < nt; ++a) {
    int32_t b = best_next[a];
    if (b >= 0 && best_prev[b] == a) {
      next[a] = b;
      prev[b] = (int32_t)a;
    }
  }
  /* chain heads: no predecessor; then the smallest index of each cycle */
  uint8_t* head = (uint8_t*)calloc(nb, 1);
  uint8_t* seen = (uint8_t*)calloc(nb, 1);
  for (int64_t i = 0; i < nt; ++i)
    if (prev[i] < 0) {
      head[i] = 1;
      for (int32_t j = (int32_t)i; j >= 0 && !seen[j]; j = next[j]) seen[j] = 1;
    }
  for (int64_t i = 0; i < nt; ++i)
    if (!seen[i]) {
      head[i] = 1;
      for (int32_t j = (int32_t)i; j >= 0 && !seen[j]; j = next[j]) seen[j] = 1;
    }
  /* prolongation of (track, end) */
  int32_t* pro_of = (int32_t*)malloc(sizeof(int32_t) * 2 * nb);
  for (int64_t i = 0; i < 2 * nt; ++i) pro_of[i] = -1;
  if (pro)
    for (int32_t k = 0; k < pro->n; ++k) pro_of[2 * pro->meta[5 * k] + pro->meta[5 * k + 1]] = k;
  /* lists, in head order */
  int64_t n_m = 0, n_c = 0;
  int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ev->n_clusters + 1));
  for (int pass = 0; pass < 2; ++pass) {
    n_m = 0;
    n_c = 0;
    int status_cap = pass == 1 && (mrg->n > mrg->cap || mrg->n_clusters > mrg->cap_clusters);
    for (int64_t h = 0; h < nt; ++h) {
      if (!head[h]) continue;
      int32_t len = 0, nseg = 0, lastseg = (int32_t)h;
      int32_t k = pro_of[2 * h];
      if (k >= 0)
        for (int32_t j = pro->meta[5 * k + 3] - 1; j >= 0; --j)
          list[len++] = pro->cluster[pro->meta[5 * k + 4] + j];
      int32_t j = (int32_t)h;
      do {
        const int32_t* m = trk->track_meta + 4 * j;
        for (int32_t q = 0; q < m[1]; ++q) list[len++] = trk->track_cluster[m[2] + q];
        if (pass == 1 && !status_cap) mrg->track_merged[j] = (int32_t)n_m;
        ++nseg;
        lastseg = j;
        j = next[j];
      } while (j >= 0 && j != h);
      k = pro_of[2 * lastseg + 1];
      if (k >= 0)
        for (int32_t q = 0; q < pro->meta[5 * k + 3]; ++q)
          list[len++] = pro->cluster[pro->meta[5 * k + 4] + q];
      if (pass == 1 && !status_cap) {
        refit_res rr;
        refit_list(ev, geo, bz, prm, len, list, &rr);
        double* P = mrg->par + 8 * n_m;
        for (int i = 0; i < 8; ++i) P[i] = rr.par[i];
        int32_t* M = mrg->meta + 5 * n_m;
        M[0] = rr.frame >= 0 ? rr.frame : ev->sector_id[slot_of[h]];
        M[1] = nseg;
        M[2] = len;
        M[3] = (int32_t)n_c;
        M[4] = (int32_t)h;
        memcpy(mrg->cluster + n_c, list, sizeof(int32_t) * (size_t)len);
      }
      ++n_m;
      n_c += len;
    }
    if (pass == 0) {
      mrg->n = (int32_t)n_m;
      mrg->n_clusters = (int32_t)n_c;
    }
  }
  int status = (mrg->n > mrg->cap || mrg->n_clusters > mrg->cap_clusters) ? 1 : 0;
  free(list); free(pro_of); free(head); free(seen); free(next); free(prev);
  free(best_next); free(best_prev); free(chi_next); free(chi_prev);
  free(first_of_slot); free(slot_of); free(e_in); free(e_out);
  return status;
}

int orc_refit(const orc_event* ev, const orc_geometry* geo, double bz, const orc_params* prm,
              int32_t n_lists, const int32_t* offsets, const int32_t* clusters, double* par,
              int32_t* frame_sector) {
  if (check_event(ev, geo) || !prm || n_lists < 0 || (n_lists > 0 && (!offsets || !par)))
    return -1;
  for (int32_t i = 0; i < n_lists; ++i) {
    refit_res rr;
    refit_list(ev, geo, bz, prm, offsets[i + 1] - offsets[i], clusters + offsets[i], &rr);
    for (int k = 0; k < 8; ++k) par[8 * i + k] = rr.par[k];
    if (frame_sector) frame_sector[i] = rr.frame;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Step-level entry points                                                   */
/* ------------------------------------------------------------------------ */

int orc_neighbours(const orc_event* ev, const orc_geometry* geo, const orc_params* prm,
                   int32_t* up, int32_t* dn) {
  if (check_event(ev, geo) || !prm || !up || !dn) return -1;
  for (int s = 0; s < ev->n_sectors; ++s) {
    sector_ctx sc;
    if (sector_init(&sc, ev, geo, prm, 0.0, s)) return -1;
    sector_neighbours(&sc, up, dn);
    sector_free(&sc);
  }
  return 0;
}

/* slot and row of cluster c, or -1 */
static int locate(const orc_event* ev, const orc_geometry* geo, int32_t c, int* row) {
  if (c < 0 || c >= ev->n_clusters) return -1;
  int64_t lo = 0, hi = (int64_t)ev->n_sectors * geo->n_rows - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (ev->row_offsets[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  *row = (int)(lo % geo->n_rows);
  return (int)(lo / geo->n_rows);
}

double orc_nf_chi2(const orc_event* ev, const orc_geometry* geo, const orc_params* prm,
                   int32_t d, int32_t c, int32_t u) {
  if (check_event(ev, geo) || !prm) return -1.0;
  int rd, rc, ru;
  int sd = locate(ev, geo, d, &rd), scn = locate(ev, geo, c, &rc), su = locate(ev, geo, u, &ru);
  if (sd < 0 || sd != scn || su != scn || rd != rc - 1 || ru != rc + 1) return -1.0;
  sector_ctx sc;
  sc.ev = ev; sc.geo = geo; sc.prm = prm; sc.bz = 0; sc.slot = scn; sc.nr = geo->n_rows;
  sc.ro = ev->row_offsets + (int64_t)scn * geo->n_rows;
  sc.sorted = NULL;
  return nf_pair_chi2(&sc, rc, d, c, u);
}

int64_t orc_seeds(const orc_event* ev, const orc_geometry* geo, const orc_params* prm,
                  const int32_t* up2, const int32_t* dn2, int32_t* seeds, int64_t cap) {
  if (check_event(ev, geo) || !prm || !up2 || !dn2) return -1;
  int64_t n = 0;
  for (int s = 0; s < ev->n_sectors; ++s) {
    sector_ctx sc;
    sc.ev = ev; sc.geo = geo; sc.prm = prm; sc.bz = 0; sc.slot = s; sc.nr = geo->n_rows;
    sc.ro = ev->row_offsets + (int64_t)s * geo->n_rows;
    sc.sorted = NULL;
    int64_t k = sector_seeds(&sc, up2, dn2, seeds ? seeds + (n < cap ? n : cap) : NULL,
                             cap - n > 0 ? cap - n : 0);
    n += k;
  }
  return (seeds && n > cap) ? -1 : n;
}

int orc_construct(const orc_event* ev, const orc_geometry* geo, double bz,
                  const orc_params* prm, const int32_t* up2, int64_t n_seeds,
                  const int32_t* seeds, orc_tracklets* tl) {
  if (check_event(ev, geo) || !prm || !up2 || !tl || n_seeds < 0) return -1;
  const int nr = geo->n_rows;
  int cur = -1;
  sector_ctx sc;
  for (int64_t t = 0; t < n_seeds; ++t) {
    int row;
    int s = locate(ev, geo, seeds[t], &row);
    if (s < 0) {
      if (cur >= 0) sector_free(&sc);
      return -1;
    }
    if (s != cur) {
      if (cur >= 0) sector_free(&sc);
      if (sector_init(&sc, ev, geo, prm, bz, s)) return -1;
      cur = s;
    }
    tl_result res;
    build_tracklet(&sc, up2, seeds[t], tl->hits + t * nr, &res);
    tl->row_lo[t] = res.row_lo;
    tl->row_hi[t] = res.row_hi;
    tl->n[t] = res.n;
    tl->ndf[t] = res.ndf;
    tl->chi2[t] = res.chi2;
    memcpy(tl->par + 6 * t, res.par, sizeof(res.par));
  }
  if (cur >= 0) sector_free(&sc);
  return 0;
}

int orc_select(const orc_event* ev, const orc_geometry* geo, double bz, const orc_params* prm,
               int64_t n_tl, const int32_t* ids, const orc_tracklets* tl, const double* weights,
               int32_t* owner, int32_t* keep) {
  if (check_event(ev, geo) || !prm || !tl || !owner || !keep || n_tl < 0) return -1;
  select_core(prm, bz, geo->n_rows, n_tl, ids, tl->hits, tl->row_lo, tl->row_hi, tl->n,
              tl->chi2, tl->ndf, tl->par, weights, 0, ev->n_clusters, owner, keep);
  return 0;
}

int orc_propagate(double x1, double* st, double* cov, double x2, double bz, double max_sinphi,
                  double* jac) {
  if (!st || !cov) return -1;
  kstate s;
  s.x = x1;
  memcpy(s.p, st, sizeof(s.p));
  memcpy(s.C, cov, sizeof(s.C));
  double J[5][5];
  if (kprop(&s, x2, bz, max_sinphi, J)) return 1;
  memcpy(st, s.p, sizeof(s.p));
  memcpy(cov, s.C, sizeof(s.C));
  if (jac) memcpy(jac, J, sizeof(J));
  return 0;
}

int orc_fit_hits(int32_t n, const double* x, const double* y, const double* z, double bz,
                 const orc_params* prm, double* st, double* cov, double* chi2,
                 int32_t* ndf) {
  if (n < 3 || !x || !y || !z || !prm || !st || !cov || !chi2 || !ndf) return -1;
  const double sy2 = prm->sigma_y * prm->sigma_y, sz2 = prm->sigma_z * prm->sigma_z;
  kstate s;
  int ns = n < prm->seed_window ? n : prm->seed_window;
  if (ns < 2) ns = 2;
  int b = ns / 2, es = ns - 1, e = n - 1;
  kseed(&s, x[0], y[0], z[0], x[b], y[b], x[es], y[es], z[es], bz, prm);
  if (fabs(s.p[2]) > prm->max_sinphi) return 1;
  for (int i = 1; i < n; ++i) {
    if (kprop(&s, x[i], bz, prm->max_sinphi, NULL)) return 1;
    kupdate(&s, y[i], z[i], sy2, sz2);
  }
  kstate w;
  w.x = x[e];
  w.p[0] = y[e];
  w.p[1] = z[e];
  w.p[2] = s.p[2];
  w.p[3] = s.p[3];
  w.p[4] = s.p[4];
  kreset_cov(&w, prm);
  double c2 = 0.0;
  for (int i = e - 1; i >= 0; --i) {
    if (kprop(&w, x[i], bz, prm->max_sinphi, NULL)) return 1;
    c2 += kupdate(&w, y[i], z[i], sy2, sz2);
  }
  memcpy(st, w.p, sizeof(w.p));
  memcpy(cov, w.C, sizeof(w.C));
  *chi2 = c2;
  *ndf = 2 * n - 5;
  return 0;
}
