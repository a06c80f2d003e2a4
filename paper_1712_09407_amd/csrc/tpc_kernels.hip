// HIP kernels (gfx950, wave64) of the TPC sector tracker.
//
// Method: Rohr et al., "ALICE HLT TPC Tracking of Pb-Pb Events on GPUs",
// section 1 (neighbours finder, evolution step, chains -> tracklets,
// tracklet construction, tracklet selection), section 3.1 (cluster weight
// w = n (alpha - chi^2/beta)), section 3.2 (sorted output).
//
// Kernels, in launch order (one event):
//   k_zero        clear the per-event counters
//   k_grid        per row slot: validate offsets, counting-sort the row into a
//                 y/z bin grid (the "initialization" of section 2, done on the
//                 device), clear the owner keys and cluster->track output
//   k_nf          per row slot: stage rows k-1 and k+1 in LDS, best straight
//                 neighbour pair of every cluster of row k
//   k_evo         per row slot: keep reciprocal links, flag chain starts of
//                 at least min_seed_len clusters, count them per row
//   k_scan_rows   one block: exclusive scan of the per-row seed counts
//   k_seed_write  per row slot: ordered compaction of chain starts (the
//                 tracklet id is the start cluster's index, so seeds come out
//                 sorted)
//   k_construct   one lane per tracklet: FP32 Kalman filter in registers,
//                 exact helix steps row by row, grid search with a chi^2 gate
//   k_assign      one lane per tracklet: weight, 64-bit atomicMax owner key
//                 per cluster (order-free, smaller id wins ties)
//   k_select      one lane per tracklet: owned clusters, >= min_clusters cut
//   k_scan_tl     one block: track index and cluster offset of kept tracklets
//   k_output      one lane per tracklet: tracks, cluster lists, cluster->track
//
// No step depends on the order in which lanes or blocks run: every choice is
// the minimum of (value, index) and every list is built by prefix sums.
#include <hip/hip_runtime.h>
#include <math.h>

#include "tpc_internal.h"

namespace tpc {

constexpr int kGridBlock = 256;
constexpr int kMaxBins = 4096;   // bins per row (LDS counting sort)
constexpr int kNfLds = 1024;     // clusters per neighbour row staged in LDS
constexpr int kScanBlock = 1024;
constexpr int kTlBlock = 64;     // one wave per block for per-tracklet kernels

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Exact decision of |a - b| <= w for finite a, b and w > 0: the rounded
// difference is corrected by its TwoSum error, so no rounding can flip it.
__device__ __forceinline__ bool within(float a, float b, float w) {
  float s = a - b;
  float bb = s - a;
  float err = (a - (s - bb)) + (-b - bb);
  float as = fabsf(s);
  float ae = s < 0.f ? -err : err;  // |a - b| = as + ae exactly
  if (as < 0.5f * w || as > 2.0f * w) return as <= w;
  float d = as - w;  // exact (Sterbenz)
  return d <= -ae;
}

__device__ __forceinline__ int bin_y(const RowGrid& g, float y) {
  float t = (y - g.y0) * g.iby;
  t = fminf(fmaxf(t, 0.f), (float)(g.ny - 1));
  return (int)t;
}
__device__ __forceinline__ int bin_z(const RowGrid& g, float z) {
  float t = (z - g.z0) * g.ibz;
  t = fminf(fmaxf(t, 0.f), (float)(g.nz - 1));
  return (int)t;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive block scan of one value per thread; s_w holds BS/64 ints.
template <int BS>
__device__ __forceinline__ int block_excl_scan(int v, int* s_w, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) {
    int t = s_w[i];
    woff += (i < w) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return woff + inc - v;
}

__device__ __forceinline__ bool event_bad(const int32_t* counters) {
  return (__builtin_nontemporal_load(&counters[C_ERR]) & (E_OFFSETS | E_NONFINITE)) != 0;
}

// ------------------------------------------------------------------ k_zero

__global__ void k_zero(int32_t* counters) {
  if (threadIdx.x < C_COUNT) counters[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ k_grid

__global__ __launch_bounds__(kGridBlock) void k_grid(DevEvent ev, KParams kp, Scratch sc,
                                                     int32_t* cluster_track) {
  __shared__ int s_cnt[kMaxBins + 1];
  __shared__ float s_red[2][kGridBlock / 64];
  __shared__ int s_w[kGridBlock / 64];
  const int rs = blockIdx.x;
  const int R = ev.n_sectors * kp.n_rows;
  const int N = ev.n_clusters;
  const int tid = threadIdx.x;
  int b = ev.ro[rs], e = ev.ro[rs + 1];
  bool bad = b < 0 || e < b || e > N || (rs == 0 && b != 0) || (rs == R - 1 && e != N);
  if (bad) {
    if (tid == 0) atomicOr(&sc.counters[C_ERR], E_OFFSETS);
    return;
  }
  const int n = e - b;
  const int r = rs % kp.n_rows;
  // z range of the row (min/max), non-finite values flagged
  float zmin = INFINITY, zmax = -INFINITY;
  int nonfin = 0;
  for (int i = b + tid; i < e; i += kGridBlock) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) {
      ++nonfin;
      continue;
    }
    zmin = fminf(zmin, z);
    zmax = fmaxf(zmax, z);
    sc.own[i] = 0ull;
    if (cluster_track) cluster_track[i] = -1;
  }
  if (nonfin) {
    atomicAdd(&sc.counters[C_NONFINITE], nonfin);
    atomicOr(&sc.counters[C_ERR], E_NONFINITE);
  }
  for (int d = 32; d >= 1; d >>= 1) {
    zmin = fminf(zmin, __shfl_xor(zmin, d, 64));
    zmax = fmaxf(zmax, __shfl_xor(zmax, d, 64));
  }
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = zmin;
    s_red[1][tid >> 6] = zmax;
  }
  __syncthreads();
  zmin = s_red[0][0];
  zmax = s_red[1][0];
  for (int i = 1; i < kGridBlock / 64; ++i) {
    zmin = fminf(zmin, s_red[0][i]);
    zmax = fmaxf(zmax, s_red[1][i]);
  }
  // bin layout: about one cluster per bin, aspect following the row's extent
  const float hw = kp.row_x[r] * kp.tan_half;
  RowGrid g;
  g.y0 = -hw;
  float wy = 2.f * hw;
  float wz = zmax - zmin;
  if (!(wz > 1e-3f)) wz = 1e-3f;
  g.z0 = (n > 0 && isfinite(zmin)) ? zmin : 0.f;
  int nbt = n < 1 ? 1 : (n > kMaxBins ? kMaxBins : n);
  int ny = clampi((int)(sqrtf((float)nbt * wy / wz) + 0.5f), 1, nbt);
  int nz = clampi(nbt / ny, 1, nbt);
  g.ny = ny;
  g.nz = nz;
  g.iby = (float)ny / wy;
  g.ibz = (float)nz / wz;
  g.bin_base = b + rs;
  g.n = n;
  const int nb = ny * nz;
  if (tid == 0) sc.grid[rs] = g;
  if (n == 0) return;  // searches test g.n first; an empty row owns no bins
  // counting sort into the bins
  for (int k = tid; k <= nb; k += kGridBlock) s_cnt[k] = 0;
  __syncthreads();
  for (int i = b + tid; i < e; i += kGridBlock) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) continue;
    atomicAdd(&s_cnt[bin_z(g, z) * ny + bin_y(g, y)], 1);
  }
  __syncthreads();
  {  // exclusive scan of s_cnt[0..nb) in place, each thread a contiguous piece
    const int per = (nb + kGridBlock - 1) / kGridBlock;
    const int lo = tid * per, hi = min(lo + per, nb);
    int sum = 0;
    for (int k = lo; k < hi; ++k) sum += s_cnt[k];
    int tot;
    int off = block_excl_scan<kGridBlock>(sum, s_w, &tot);
    for (int k = lo; k < hi; ++k) {
      int v = s_cnt[k];
      s_cnt[k] = off;
      off += v;
    }
    __syncthreads();
    if (tid == 0) s_cnt[nb] = tot;
    __syncthreads();
  }
  for (int k = tid; k <= nb; k += kGridBlock) sc.bins[g.bin_base + k] = s_cnt[k];
  __syncthreads();
  for (int i = b + tid; i < e; i += kGridBlock) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) continue;
    int pos = atomicAdd(&s_cnt[bin_z(g, z) * ny + bin_y(g, y)], 1);
    sc.g_yz[b + pos] = make_float2(y, z);
    sc.g_id[b + pos] = i;
  }
}

// ------------------------------------------------------------------ k_nf

// Neighbour-row view (LDS or global).
struct RowView {
  const float2* yz;
  const int32_t* id;
  const int32_t* bins;  // bins of the row, index 0 = first bin
  RowGrid g;
};

// Best (chi2, d, u) pair for a cluster at (yc, zc) of row k (section 1).
__device__ __forceinline__ void nf_search(const RowView& D, const RowView& U, float yc, float zc,
                                          float t, float wy, float wz, float isy2, float isz2,
                                          float inorm, float& best, int& bd, int& bu) {
  const float m = 1e-3f;  // bin ranges are only an accelerator: widen them
  const int dy0 = bin_y(D.g, yc - wy - m), dy1 = bin_y(D.g, yc + wy + m);
  const int dz0 = bin_z(D.g, zc - wz - m), dz1 = bin_z(D.g, zc + wz + m);
  const int uy0 = bin_y(U.g, yc - wy - m), uy1 = bin_y(U.g, yc + wy + m);
  const int uz0 = bin_z(U.g, zc - wz - m), uz1 = bin_z(U.g, zc + wz + m);
  for (int iz = dz0; iz <= dz1; ++iz) {
    const int j0 = D.bins[iz * D.g.ny + dy0], j1 = D.bins[iz * D.g.ny + dy1 + 1];
    for (int j = j0; j < j1; ++j) {
      const float2 pd = D.yz[j];
      if (!within(pd.x, yc, wy) || !within(pd.y, zc, wz)) continue;
      const int idd = D.id[j];
      const float dyd = pd.x - yc, dzd = pd.y - zc;
      for (int kz = uz0; kz <= uz1; ++kz) {
        const int k0 = U.bins[kz * U.g.ny + uy0], k1 = U.bins[kz * U.g.ny + uy1 + 1];
        for (int k = k0; k < k1; ++k) {
          const float2 pu = U.yz[k];
          if (!within(pu.x, yc, wy) || !within(pu.y, zc, wz)) continue;
          const int idu = U.id[k];
          const float ry = dyd + t * ((pu.x - yc) - dyd);
          const float rz = dzd + t * ((pu.y - zc) - dzd);
          const float chi2 = (ry * ry * isy2 + rz * rz * isz2) * inorm;
          if (bd < 0 || chi2 < best ||
              (chi2 == best && (idd < bd || (idd == bd && idu < bu)))) {
            best = chi2;
            bd = idd;
            bu = idu;
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(kGridBlock) void k_nf(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ float2 s_yz[2][kNfLds];
  __shared__ int32_t s_id[2][kNfLds];
  __shared__ int32_t s_bins[2][kNfLds + 1];
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int r = rs % kp.n_rows;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  if (r == 0 || r == kp.n_rows - 1) {
    for (int i = b + tid; i < e; i += kGridBlock) {
      sc.up[i] = -1;
      sc.dn[i] = -1;
    }
    return;
  }
  const RowGrid gd = sc.grid[rs - 1], gu = sc.grid[rs + 1];
  const int bd_ = ev.ro[rs - 1], bu_ = ev.ro[rs + 1];
  const bool stage = gd.n <= kNfLds && gu.n <= kNfLds;
  const float xd = kp.row_x[r - 1], xc = kp.row_x[r], xu = kp.row_x[r + 1];
  const float t = (xc - xd) / (xu - xd);
  const float inorm = 1.f / (1.f + t * t + (1.f - t) * (1.f - t));
  const float isy2 = 1.f / kp.sy2, isz2 = 1.f / kp.sz2;
  if (stage) {
    const int nbd = gd.ny * gd.nz, nbu = gu.ny * gu.nz;
    for (int i = tid; i < gd.n; i += kGridBlock) {
      s_yz[0][i] = sc.g_yz[bd_ + i];
      s_id[0][i] = sc.g_id[bd_ + i];
    }
    for (int i = tid; i < gu.n; i += kGridBlock) {
      s_yz[1][i] = sc.g_yz[bu_ + i];
      s_id[1][i] = sc.g_id[bu_ + i];
    }
    if (gd.n > 0)
      for (int i = tid; i <= nbd; i += kGridBlock) s_bins[0][i] = sc.bins[gd.bin_base + i];
    if (gu.n > 0)
      for (int i = tid; i <= nbu; i += kGridBlock) s_bins[1][i] = sc.bins[gu.bin_base + i];
    __syncthreads();
  }
  for (int i = b + tid; i < e; i += kGridBlock) {
    const float yc = ev.y[i], zc = ev.z[i];
    float best = INFINITY;
    int bd = -1, bu = -1;
    if (gd.n > 0 && gu.n > 0) {
      if (stage) {
        RowView D{s_yz[0], s_id[0], s_bins[0], gd}, U{s_yz[1], s_id[1], s_bins[1], gu};
        nf_search(D, U, yc, zc, t, kp.nf_win_y, kp.nf_win_z, isy2, isz2, inorm, best, bd, bu);
      } else {
        RowView D{sc.g_yz + bd_, sc.g_id + bd_, sc.bins + gd.bin_base, gd};
        RowView U{sc.g_yz + bu_, sc.g_id + bu_, sc.bins + gu.bin_base, gu};
        nf_search(D, U, yc, zc, t, kp.nf_win_y, kp.nf_win_z, isy2, isz2, inorm, best, bd, bu);
      }
    }
    const bool ok = bd >= 0 && best <= kp.nf_chi2_max;
    sc.up[i] = ok ? bu : -1;
    sc.dn[i] = ok ? bd : -1;
  }
}

// ------------------------------------------------------------------ k_evo

__global__ __launch_bounds__(kGridBlock) void k_evo(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ int s_w[kGridBlock / 64];
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  int cnt = 0;
  for (int i = b + tid; i < e; i += kGridBlock) {
    const int u = sc.up[i], d = sc.dn[i];
    const int u2 = (u >= 0 && sc.dn[u] == i) ? u : -1;
    const int d2 = (d >= 0 && sc.up[d] == i) ? d : -1;
    sc.up2[i] = u2;
    sc.dn2[i] = d2;
    bool start = d2 < 0 && u2 >= 0;
    if (start) {
      // chain length >= min_seed_len: follow reciprocal links outward
      int len = 2, cur = u2;
      while (len < kp.min_seed_len) {
        const int nu = sc.up[cur];
        if (nu < 0 || sc.dn[nu] != cur) break;
        cur = nu;
        ++len;
      }
      start = len >= kp.min_seed_len;
    }
    sc.start[i] = start ? 1 : 0;
    cnt += start ? 1 : 0;
  }
  int tot;
  block_excl_scan<kGridBlock>(cnt, s_w, &tot);
  if (tid == 0) sc.row_cnt[rs] = tot;
}

// ------------------------------------------------------------------ scans

__global__ __launch_bounds__(kScanBlock) void k_scan_rows(int R, Scratch sc) {
  __shared__ int s_w[kScanBlock / 64];
  if (event_bad(sc.counters)) return;
  const int tid = threadIdx.x;
  int carry = 0;
  for (int base = 0; base < R; base += kScanBlock) {
    const int i = base + tid;
    const int v = i < R ? sc.row_cnt[i] : 0;
    int tot;
    const int ex = block_excl_scan<kScanBlock>(v, s_w, &tot);
    if (i < R) sc.row_cnt[i] = carry + ex;
    carry += tot;
  }
  if (tid == 0) {
    sc.row_cnt[R] = carry;
    sc.counters[C_SEEDS] = carry;
    if (carry > sc.cap_tl) atomicOr(&sc.counters[C_ERR], E_TL_OVERFLOW);
  }
}

__global__ __launch_bounds__(kGridBlock) void k_seed_write(DevEvent ev, Scratch sc) {
  __shared__ int s_w[kGridBlock / 64];
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  int base = sc.row_cnt[rs];
  if (sc.row_cnt[rs + 1] == base) return;  // uniform: no start in this row
  for (int c0 = b; c0 < e; c0 += kGridBlock) {
    const int i = c0 + tid;
    const int f = (i < e) ? sc.start[i] : 0;
    int tot;
    const int rank = block_excl_scan<kGridBlock>(f, s_w, &tot);
    if (f && base + rank < sc.cap_tl) {
      sc.seeds[base + rank] = i;
      sc.seed_rs[base + rank] = rs;
    }
    base += tot;
  }
}

// ------------------------------------------------------------------ track model

// Lower-triangular packed symmetric 5x5 covariance.
struct Cov {
  float c00, c10, c11, c20, c21, c22, c30, c31, c32, c33, c40, c41, c42, c43, c44;
};

struct KState {
  float x, y, z, sp, tl, qpt;
  Cov C;
};

__device__ __forceinline__ void reset_cov(Cov& C, const KParams& kp) {
  C.c00 = kp.sy2;
  C.c11 = kp.sz2;
  C.c22 = kp.prior_sinphi;
  C.c33 = kp.prior_tanl;
  C.c44 = kp.prior_qpt;
  C.c10 = C.c20 = C.c21 = C.c30 = C.c31 = C.c32 = C.c40 = C.c41 = C.c42 = C.c43 = 0.f;
}

// asin(u)/u and its derivative; series below |u| = 0.1 (next term < 1e-9).
__device__ __forceinline__ float asinc(float u) {
  const float u2 = u * u;
  if (u2 < 0.01f) return 1.f + u2 * (1.f / 6.f + u2 * (3.f / 40.f + u2 * (5.f / 112.f)));
  return asinf(u) / u;
}
__device__ __forceinline__ float asinc_d(float u, float isq) {
  const float u2 = u * u;
  if (u2 < 0.01f) return u * (1.f / 3.f + u2 * (3.f / 10.f + u2 * (15.f / 56.f)));
  return (u * isq - asinf(u)) / u2;
}

// Exact helix step to x2 with the analytic Jacobian (section 1's Kalman fit
// needs the extrapolation to adjacent rows).  Returns false, leaving the
// state unchanged, if |sin phi| would pass max_sinphi.
__device__ __forceinline__ bool propagate(KState& s, float x2, const KParams& kp) {
  const float k = kp.k_curv;
  const float dx = x2 - s.x;
  const float kap = k * s.qpt;
  const float s1 = s.sp, s2 = s1 - kap * dx;
  if (fabsf(s1) > kp.max_sinphi || fabsf(s2) > kp.max_sinphi) return false;
  const float c1 = sqrtf((1.f - s1) * (1.f + s1)), c2 = sqrtf((1.f - s2) * (1.f + s2));
  const float ic1 = 1.f / c1, ic2 = 1.f / c2;
  const float T = (s1 + s2) / (c1 + c2);
  const float Q2 = 1.f + T * T;
  const float Q = sqrtf(Q2);
  const float u = 0.5f * kap * dx * Q;
  const float isq = 1.f / sqrtf(1.f - u * u);
  const float h = asinc(u);
  const float ds = dx * Q * h;
  const float dT_ds1 = 0.5f * Q2 * (ic1 + ic2);
  const float dT_dk = -0.5f * Q2 * dx * ic2;
  const float TQ = T / Q;
  const float dds_ds1 = dx * TQ * dT_ds1 * isq;
  const float dds_dk = dx * (TQ * dT_dk * isq + 0.5f * Q2 * dx * asinc_d(u, isq));
  const float a = dx * dT_ds1;        // dy/dsinphi
  const float bq = dx * dT_dk * k;    // dy/dqpt
  const float c = s.tl * dds_ds1;     // dz/dsinphi
  const float d = ds;                 // dz/dtanl
  const float ee = s.tl * dds_dk * k; // dz/dqpt
  const float f = -dx * k;            // dsinphi/dqpt
  Cov& C = s.C;
  // T = J C (rows 0..2 differ from C)
  const float t00 = C.c00 + a * C.c20 + bq * C.c40;
  const float t02 = C.c20 + a * C.c22 + bq * C.c42;
  const float t04 = C.c40 + a * C.c42 + bq * C.c44;
  const float t10 = C.c10 + c * C.c20 + d * C.c30 + ee * C.c40;
  const float t11 = C.c11 + c * C.c21 + d * C.c31 + ee * C.c41;
  const float t12 = C.c21 + c * C.c22 + d * C.c32 + ee * C.c42;
  const float t13 = C.c31 + c * C.c32 + d * C.c33 + ee * C.c43;
  const float t14 = C.c41 + c * C.c42 + d * C.c43 + ee * C.c44;
  const float t20 = C.c20 + f * C.c40;
  const float t21 = C.c21 + f * C.c41;
  const float t22 = C.c22 + f * C.c42;
  const float t23 = C.c32 + f * C.c43;
  const float t24 = C.c42 + f * C.c44;
  Cov N;
  N.c00 = t00 + a * t02 + bq * t04;
  N.c10 = t10 + a * t12 + bq * t14;
  N.c11 = t11 + c * t12 + d * t13 + ee * t14;
  N.c20 = t20 + a * t22 + bq * t24;
  N.c21 = t21 + c * t22 + d * t23 + ee * t24;
  N.c22 = t22 + f * t24;
  N.c30 = C.c30 + a * C.c32 + bq * C.c43;
  N.c31 = C.c31 + c * C.c32 + d * C.c33 + ee * C.c43;
  N.c32 = C.c32 + f * C.c43;
  N.c33 = C.c33;
  N.c40 = C.c40 + a * C.c42 + bq * C.c44;
  N.c41 = C.c41 + c * C.c42 + d * C.c43 + ee * C.c44;
  N.c42 = C.c42 + f * C.c44;
  N.c43 = C.c43;
  N.c44 = C.c44;
  C = N;
  s.y += dx * T;
  s.z += s.tl * ds;
  s.sp = s2;
  s.x = x2;
  return true;
}

// Kalman update with the measurement (my, mz); returns its chi^2.
__device__ __forceinline__ float kf_update(KState& s, float my, float mz, const KParams& kp) {
  Cov& C = s.C;
  const float S00 = C.c00 + kp.sy2, S01 = C.c10, S11 = C.c11 + kp.sz2;
  const float idet = 1.f / (S00 * S11 - S01 * S01);
  const float i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
  const float ry = my - s.y, rz = mz - s.z;
  const float chi2 = ry * ry * i00 + 2.f * ry * rz * i01 + rz * rz * i11;
  // K = C H^T S^-1 (columns 0 and 1 of C)
  const float k00 = C.c00 * i00 + C.c10 * i01, k01 = C.c00 * i01 + C.c10 * i11;
  const float k10 = C.c10 * i00 + C.c11 * i01, k11 = C.c10 * i01 + C.c11 * i11;
  const float k20 = C.c20 * i00 + C.c21 * i01, k21 = C.c20 * i01 + C.c21 * i11;
  const float k30 = C.c30 * i00 + C.c31 * i01, k31 = C.c30 * i01 + C.c31 * i11;
  const float k40 = C.c40 * i00 + C.c41 * i01, k41 = C.c40 * i01 + C.c41 * i11;
  s.y += k00 * ry + k01 * rz;
  s.z += k10 * ry + k11 * rz;
  s.sp += k20 * ry + k21 * rz;
  s.tl += k30 * ry + k31 * rz;
  s.qpt += k40 * ry + k41 * rz;
  // C -= K (H C): rows 0 and 1 of the old C
  const float h00 = C.c00, h01 = C.c10, h02 = C.c20, h03 = C.c30, h04 = C.c40;
  const float h10 = C.c10, h11 = C.c11, h12 = C.c21, h13 = C.c31, h14 = C.c41;
  C.c00 -= k00 * h00 + k01 * h10;
  C.c10 -= k10 * h00 + k11 * h10;
  C.c11 -= k10 * h01 + k11 * h11;
  C.c20 -= k20 * h00 + k21 * h10;
  C.c21 -= k20 * h01 + k21 * h11;
  C.c22 -= k20 * h02 + k21 * h12;
  C.c30 -= k30 * h00 + k31 * h10;
  C.c31 -= k30 * h01 + k31 * h11;
  C.c32 -= k30 * h02 + k31 * h12;
  C.c33 -= k30 * h03 + k31 * h13;
  C.c40 -= k40 * h00 + k41 * h10;
  C.c41 -= k40 * h01 + k41 * h11;
  C.c42 -= k40 * h02 + k41 * h12;
  C.c43 -= k40 * h03 + k41 * h13;
  C.c44 -= k40 * h04 + k41 * h14;
  return chi2;
}

// Seed from clusters a (first), b (middle), e (last) of the chain: the circle
// through them in (x, y) gives curvature and direction at a; tan lambda is
// the z rise over the arc a -> e.
__device__ __forceinline__ void seed3(KState& s, float xa, float ya, float za, float xb, float yb,
                                      float xe, float ye, float ze, const KParams& kp) {
  const float d1x = xb - xa, d1y = yb - ya, d2x = xe - xa, d2y = ye - ya;
  float kappa = 0.f;
  if (kp.bz != 0.f) {
    const float cross = d1x * d2y - d1y * d2x;
    const float den = sqrtf(d1x * d1x + d1y * d1y) * sqrtf(d2x * d2x + d2y * d2y) *
                      sqrtf((d2x - d1x) * (d2x - d1x) + (d2y - d1y) * (d2y - d1y));
    kappa = den > 0.f ? -2.f * cross / den : 0.f;
  }
  const float L = sqrtf(d2x * d2x + d2y * d2y);
  float u = 0.5f * kappa * L;
  u = fminf(fmaxf(u, -1.f), 1.f);
  s.x = xa;
  s.y = ya;
  s.z = za;
  s.sp = (d2y / L) * sqrtf(1.f - u * u) + (d2x / L) * u;
  s.tl = (ze - za) / (L * asinc(u));
  s.qpt = kp.bz != 0.f ? kappa / kp.k_curv : 0.f;
  reset_cov(s.C, kp);
}

// Work done by one lane of the constructor (for the algorithmic FLOP count).
struct Work {
  int steps = 0, updates = 0, cands = 0;
};

// Best cluster of a row inside the chi^2 gate (smallest (chi2, index)).
__device__ __forceinline__ int search_row(const Scratch& sc, const RowGrid& g, int rb,
                                          const KState& s, const KParams& kp, float& chi2_out,
                                          Work& wk) {
  if (g.n == 0) return -1;
  const float S00 = s.C.c00 + kp.sy2, S01 = s.C.c10, S11 = s.C.c11 + kp.sz2;
  const float idet = 1.f / (S00 * S11 - S01 * S01);
  const float wy = sqrtf(kp.chi2_gate * S00) * 1.0001f + 1e-4f;
  const float wz = sqrtf(kp.chi2_gate * S11) * 1.0001f + 1e-4f;
  const int iy0 = bin_y(g, s.y - wy), iy1 = bin_y(g, s.y + wy);
  const int iz0 = bin_z(g, s.z - wz), iz1 = bin_z(g, s.z + wz);
  float best = INFINITY;
  int bid = -1;
  for (int iz = iz0; iz <= iz1; ++iz) {
    const int j0 = sc.bins[g.bin_base + iz * g.ny + iy0];
    const int j1 = sc.bins[g.bin_base + iz * g.ny + iy1 + 1];
    wk.cands += j1 - j0;
    for (int j = j0; j < j1; ++j) {
      const float2 v = sc.g_yz[rb + j];
      const float ry = v.x - s.y, rz = v.y - s.z;
      const float chi2 = (ry * ry * S11 - 2.f * ry * rz * S01 + rz * rz * S00) * idet;
      if (chi2 <= kp.chi2_gate) {
        const int id = sc.g_id[rb + j];
        if (chi2 < best || (chi2 == best && id < bid)) {
          best = chi2;
          bid = id;
        }
      }
    }
  }
  chi2_out = best;
  return bid;
}

// One extension row: 0 = cluster collected, 1 = miss, 2 = stop.
__device__ __forceinline__ int extend_step(const DevEvent& ev, const Scratch& sc, const KParams& kp,
                                           const float* s_x, int rsb, int r, KState& s, int& hit,
                                           float& chi2, Work& wk) {
  if (!propagate(s, s_x[r], kp)) return 2;
  ++wk.steps;
  if (fabsf(s.z) > kp.z_max) return 2;
  if (fabsf(s.y) > s_x[r] * kp.tan_half) return 1;
  const RowGrid g = sc.grid[rsb + r];
  float c2;
  const int j = search_row(sc, g, ev.ro[rsb + r], s, kp, c2, wk);
  if (j < 0) return 1;
  chi2 = kf_update(s, ev.y[j], ev.z[j], kp);
  ++wk.updates;
  hit = j;
  return 0;
}

// ------------------------------------------------------------------ k_construct

__global__ __launch_bounds__(kTlBlock) void k_construct(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ float s_x[TPC_MAX_ROWS];
  if (event_bad(sc.counters)) return;
  for (int i = threadIdx.x; i < kp.n_rows; i += kTlBlock) s_x[i] = kp.row_x[i];
  __syncthreads();
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int nr = kp.n_rows;
  Work wk;
  for (int t = blockIdx.x * kTlBlock + threadIdx.x; t < n_tl; t += gridDim.x * kTlBlock) {
    const int start = sc.seeds[t];
    const int rs0 = sc.seed_rs[t];
    const int k0 = rs0 % nr;
    const int rsb = rs0 - k0;
    int32_t* H = sc.hits + (size_t)t * kHitStride;
    // the chain of one-to-one links
    int m = 0, last = start;
    for (int c = start; c >= 0 && k0 + m < nr; c = sc.up2[c]) {
      H[k0 + m] = c;
      last = c;
      ++m;
    }
    const int bmid = H[k0 + m / 2];
    KState s;
    seed3(s, s_x[k0], ev.y[start], ev.z[start], s_x[k0 + m / 2], ev.y[bmid], s_x[k0 + m - 1],
          ev.y[last], ev.z[last], kp);
    bool dropped = fabsf(s.sp) > kp.max_sinphi;
    int last_row = k0;
    float l_sp = s.sp, l_tl = s.tl, l_q = s.qpt;
    // outward filter through the chain, unconditionally
    for (int j = 1; j < m && !dropped; ++j) {
      if (!propagate(s, s_x[k0 + j], kp)) {
        dropped = true;
        break;
      }
      const int c = H[k0 + j];
      kf_update(s, ev.y[c], ev.z[c], kp);
      wk.steps += 1;
      wk.updates += 1;
      last_row = k0 + j;
      l_sp = s.sp;
      l_tl = s.tl;
      l_q = s.qpt;
    }
    // outward extension
    if (!dropped) {
      int misses = 0;
      for (int r = k0 + m; r < nr; ++r) {
        int h = -1;
        float c2;
        const int st = extend_step(ev, sc, kp, s_x, rsb, r, s, h, c2, wk);
        if (st == 2) break;
        H[r] = h;
        if (st == 0) {
          last_row = r;
          l_sp = s.sp;
          l_tl = s.tl;
          l_q = s.qpt;
          misses = 0;
        } else if (++misses > kp.max_miss) {
          break;
        }
      }
    }
    // inward refit from the outermost collected cluster with a fresh covariance
    int n = 0, inner = 0, ndf = 0;
    float chi2 = 0.f;
    float ox = 0.f, oy = 0.f, oz = 0.f, osp = 0.f, otl = 0.f, oq = 0.f;
    if (!dropped) {
      const int ho = H[last_row];
      KState w;
      w.x = s_x[last_row];
      w.y = ev.y[ho];
      w.z = ev.z[ho];
      w.sp = l_sp;
      w.tl = l_tl;
      w.qpt = l_q;
      reset_cov(w.C, kp);
      n = 1;
      inner = last_row;
      ox = w.x; oy = w.y; oz = w.z; osp = w.sp; otl = w.tl; oq = w.qpt;
      for (int r = last_row - 1; r >= k0; --r) {
        if (!propagate(w, s_x[r], kp)) {
          dropped = true;
          break;
        }
        ++wk.steps;
        const int c = H[r];
        if (c >= 0) {
          ++wk.updates;
          chi2 += kf_update(w, ev.y[c], ev.z[c], kp);
          ++n;
          inner = r;
          ox = w.x; oy = w.y; oz = w.z; osp = w.sp; otl = w.tl; oq = w.qpt;
        }
      }
      if (!dropped) {
        int misses = 0;
        for (int r = k0 - 1; r >= 0; --r) {
          int h = -1;
          float c2 = 0.f;
          const int st = extend_step(ev, sc, kp, s_x, rsb, r, w, h, c2, wk);
          if (st == 2) break;
          H[r] = h;
          if (st == 0) {
            chi2 += c2;
            ++n;
            inner = r;
            ox = w.x; oy = w.y; oz = w.z; osp = w.sp; otl = w.tl; oq = w.qpt;
            misses = 0;
          } else if (++misses > kp.max_miss) {
            break;
          }
        }
      }
      ndf = 2 * n - 5;
    }
    if (dropped) {
      n = 0;
      ndf = 0;
      chi2 = 0.f;
      sc.row_lo[t] = 0;
      sc.row_hi[t] = -1;
    } else {
      sc.row_lo[t] = inner;
      sc.row_hi[t] = last_row;
    }
    sc.n[t] = n;
    sc.ndf[t] = ndf;
    sc.chi2[t] = chi2;
    float* P = sc.par + (size_t)t * 6;
    P[0] = ox; P[1] = oy; P[2] = oz; P[3] = osp; P[4] = otl; P[5] = oq;
  }
  // one atomic per wave and counter
  int st = wk.steps, up = wk.updates, ca = wk.cands;
  for (int d = 32; d >= 1; d >>= 1) {
    st += __shfl_xor(st, d, 64);
    up += __shfl_xor(up, d, 64);
    ca += __shfl_xor(ca, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&sc.counters[C_STEPS], st);
    atomicAdd(&sc.counters[C_UPDATES], up);
    atomicAdd(&sc.counters[C_CANDS], ca);
  }
}

// ------------------------------------------------------------------ selection

__device__ __forceinline__ unsigned int order_bits(float w) {
  const unsigned int u = __float_as_uint(w + 0.f);  // -0 -> +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(kTlBlock) void k_assign(KParams kp, Scratch sc) {
  if (event_bad(sc.counters)) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  for (int t = blockIdx.x * kTlBlock + threadIdx.x; t < n_tl; t += gridDim.x * kTlBlock) {
    const int n = sc.n[t];
    const float qpt = sc.par[(size_t)t * 6 + 5];
    unsigned long long key = 0ull;
    if (n >= kp.min_clusters && (kp.bz == 0.f || fabsf(qpt) <= kp.max_qpt)) {
      const float w = (float)n * (kp.alpha - (sc.chi2[t] / (float)sc.ndf[t]) / kp.beta);
      key = ((unsigned long long)order_bits(w) << 32) |
            (unsigned long long)(0xFFFFFFFFu - (unsigned int)sc.seeds[t]);
      const int32_t* H = sc.hits + (size_t)t * kHitStride;
      for (int r = sc.row_lo[t]; r <= sc.row_hi[t]; ++r) {
        const int c = H[r];
        if (c >= 0) atomicMax(&sc.own[c], key);
      }
    }
    sc.key[t] = key;
  }
}

__global__ __launch_bounds__(kTlBlock) void k_select(KParams kp, Scratch sc) {
  if (event_bad(sc.counters)) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  for (int t = blockIdx.x * kTlBlock + threadIdx.x; t < n_tl; t += gridDim.x * kTlBlock) {
    const unsigned long long key = sc.key[t];
    int owned = 0;
    if (key != 0ull) {
      const int32_t* H = sc.hits + (size_t)t * kHitStride;
      for (int r = sc.row_lo[t]; r <= sc.row_hi[t]; ++r) {
        const int c = H[r];
        owned += (c >= 0 && sc.own[c] == key) ? 1 : 0;
      }
    }
    const bool kept = owned >= kp.min_clusters;
    sc.kept[t] = kept ? 1 : 0;
    sc.owned[t] = kept ? owned : 0;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tl(Scratch sc, int cap_tracks,
                                                        int cap_track_clusters) {
  __shared__ int s_w[kScanBlock / 64];
  if (event_bad(sc.counters)) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int tid = threadIdx.x;
  int carry_t = 0, carry_c = 0;
  for (int base = 0; base < n_tl; base += kScanBlock) {
    const int i = base + tid;
    const int k = i < n_tl ? sc.kept[i] : 0;
    const int o = i < n_tl ? sc.owned[i] : 0;
    int tt, tc;
    const int et = block_excl_scan<kScanBlock>(k, s_w, &tt);
    const int ec = block_excl_scan<kScanBlock>(o, s_w, &tc);
    if (i < n_tl) {
      sc.trk_idx[i] = carry_t + et;
      sc.trk_off[i] = carry_c + ec;
    }
    carry_t += tt;
    carry_c += tc;
  }
  if (tid == 0) {
    sc.counters[C_TRACKS] = carry_t;
    sc.counters[C_TRACK_CLUSTERS] = carry_c;
    if (carry_t > cap_tracks || carry_c > cap_track_clusters)
      atomicOr(&sc.counters[C_ERR], E_CAPACITY);
  }
}

__global__ __launch_bounds__(kTlBlock) void k_output(DevEvent ev, KParams kp, Scratch sc,
                                                     Outputs out) {
  if (__builtin_nontemporal_load(&sc.counters[C_ERR]) != 0) {
    // bad input, capacity exceeded or tracklet overflow: nothing is written
    return;
  }
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  for (int t = blockIdx.x * kTlBlock + threadIdx.x; t < n_tl; t += gridDim.x * kTlBlock) {
    if (!sc.kept[t]) continue;
    const int i = sc.trk_idx[t];
    const int off = sc.trk_off[t];
    const unsigned long long key = sc.key[t];
    const int32_t* H = sc.hits + (size_t)t * kHitStride;
    int k = 0;
    for (int r = sc.row_lo[t]; r <= sc.row_hi[t]; ++r) {
      const int c = H[r];
      if (c >= 0 && sc.own[c] == key) {
        out.track_cluster[off + k] = c;
        out.cluster_track[c] = i;
        ++k;
      }
    }
    const float* P = sc.par + (size_t)t * 6;
    float* O = out.track_par + (size_t)i * 8;
    O[0] = P[0]; O[1] = P[1]; O[2] = P[2]; O[3] = P[3]; O[4] = P[4]; O[5] = P[5];
    O[6] = sc.chi2[t];
    O[7] = (float)sc.ndf[t];
    int32_t* M = out.track_meta + (size_t)i * 4;
    M[0] = ev.sector_id[sc.seed_rs[t] / kp.n_rows];
    M[1] = k;
    M[2] = off;
    M[3] = sc.seeds[t];
  }
}

// ------------------------------------------------------------------ host side

static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t scratch_bytes(int64_t N, int64_t R, int64_t T) {
  size_t b = 0;
  b += align_up(sizeof(int32_t) * C_COUNT);
  b += align_up(sizeof(RowGrid) * R);
  b += align_up(sizeof(int32_t) * (N + R + 1));
  b += align_up(sizeof(float2) * N);
  b += align_up(sizeof(int32_t) * N) * 6;  // g_id, up, dn, up2, dn2 + start (bytes, padded)
  b += align_up(sizeof(unsigned long long) * N);
  b += align_up(sizeof(int32_t) * (R + 1));
  b += align_up(sizeof(int32_t) * T) * 2;
  b += align_up(sizeof(int32_t) * T * kHitStride);
  b += align_up(sizeof(int32_t) * T) * 4;
  b += align_up(sizeof(float) * T);
  b += align_up(sizeof(float) * T * 6);
  b += align_up(sizeof(unsigned long long) * T);
  b += align_up(sizeof(int32_t) * T) * 4;
  return b;
}

void scratch_carve(void* base, int64_t N, int64_t R, int64_t T, Scratch* sc) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align_up(bytes);
    return r;
  };
  sc->counters = (int32_t*)take(sizeof(int32_t) * C_COUNT);
  sc->grid = (RowGrid*)take(sizeof(RowGrid) * R);
  sc->bins = (int32_t*)take(sizeof(int32_t) * (N + R + 1));
  sc->g_yz = (float2*)take(sizeof(float2) * N);
  sc->g_id = (int32_t*)take(sizeof(int32_t) * N);
  sc->up = (int32_t*)take(sizeof(int32_t) * N);
  sc->dn = (int32_t*)take(sizeof(int32_t) * N);
  sc->up2 = (int32_t*)take(sizeof(int32_t) * N);
  sc->dn2 = (int32_t*)take(sizeof(int32_t) * N);
  sc->start = (uint8_t*)take(sizeof(int32_t) * N);
  sc->own = (unsigned long long*)take(sizeof(unsigned long long) * N);
  sc->row_cnt = (int32_t*)take(sizeof(int32_t) * (R + 1));
  sc->cap_tl = (int32_t)T;
  sc->seeds = (int32_t*)take(sizeof(int32_t) * T);
  sc->seed_rs = (int32_t*)take(sizeof(int32_t) * T);
  sc->hits = (int32_t*)take(sizeof(int32_t) * T * kHitStride);
  sc->row_lo = (int32_t*)take(sizeof(int32_t) * T);
  sc->row_hi = (int32_t*)take(sizeof(int32_t) * T);
  sc->n = (int32_t*)take(sizeof(int32_t) * T);
  sc->ndf = (int32_t*)take(sizeof(int32_t) * T);
  sc->chi2 = (float*)take(sizeof(float) * T);
  sc->par = (float*)take(sizeof(float) * T * 6);
  sc->key = (unsigned long long*)take(sizeof(unsigned long long) * T);
  sc->owned = (int32_t*)take(sizeof(int32_t) * T);
  sc->kept = (int32_t*)take(sizeof(int32_t) * T);
  sc->trk_idx = (int32_t*)take(sizeof(int32_t) * T);
  sc->trk_off = (int32_t*)take(sizeof(int32_t) * T);
}

// Per-tracklet kernels: enough waves for every tracklet of a large event,
// lanes stride over the rest.
static inline int tl_blocks(int64_t T) {
  int64_t b = (T + kTlBlock - 1) / kTlBlock;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

const char* const kKernelNames[K_NUM] = {
    "k_zero", "k_grid", "k_nf", "k_evo", "k_scan_rows", "k_seed_write", "k_construct",
    "k_assign", "k_select", "k_scan_tl", "k_output"};

hipError_t enqueue_event(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const Outputs& out, int upto, hipStream_t st, const KernelTimer* tm) {
  const int R = ev.n_sectors * kp.n_rows;
  auto pre = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][0], st);
  };
  auto post = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][1], st);
  };
  pre(K_ZERO);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, sc.counters);
  post(K_ZERO);
  pre(K_GRID);
  hipLaunchKernelGGL(k_grid, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc, out.cluster_track);
  post(K_GRID);
  pre(K_NF);
  hipLaunchKernelGGL(k_nf, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc);
  post(K_NF);
  pre(K_EVO);
  hipLaunchKernelGGL(k_evo, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc);
  post(K_EVO);
  if (upto <= STAGE_LINKS) return hipGetLastError();
  pre(K_SCAN_ROWS);
  hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kScanBlock), 0, st, R, sc);
  post(K_SCAN_ROWS);
  pre(K_SEED_WRITE);
  hipLaunchKernelGGL(k_seed_write, dim3(R), dim3(kGridBlock), 0, st, ev, sc);
  post(K_SEED_WRITE);
  if (upto <= STAGE_SEEDS) return hipGetLastError();
  const int nb = tl_blocks(sc.cap_tl);
  pre(K_CONSTRUCT);
  hipLaunchKernelGGL(k_construct, dim3(nb), dim3(kTlBlock), 0, st, ev, kp, sc);
  post(K_CONSTRUCT);
  if (upto <= STAGE_TRACKLETS) return hipGetLastError();
  pre(K_ASSIGN);
  hipLaunchKernelGGL(k_assign, dim3(nb), dim3(kTlBlock), 0, st, kp, sc);
  post(K_ASSIGN);
  pre(K_SELECT);
  hipLaunchKernelGGL(k_select, dim3(nb), dim3(kTlBlock), 0, st, kp, sc);
  post(K_SELECT);
  pre(K_SCAN_TL);
  hipLaunchKernelGGL(k_scan_tl, dim3(1), dim3(kScanBlock), 0, st, sc, out.cap_tracks,
                     out.cap_track_clusters);
  post(K_SCAN_TL);
  pre(K_OUTPUT);
  hipLaunchKernelGGL(k_output, dim3(nb), dim3(kTlBlock), 0, st, ev, kp, sc, out);
  post(K_OUTPUT);
  return hipGetLastError();
}

}  // namespace tpc
