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
//                 device), clear the cluster->track output
//   k_nf          per row slot (rows of all sectors in row order, the dense
//                 inner rows first): stage rows k-1 and k+1 in LDS, best
//                 straight neighbour pair of every cluster of row k
//   k_evo         per row slot: keep reciprocal links, flag chain starts of
//                 at least min_seed_len clusters, count them per row
//   k_rows_reduce, exclusive scan of the per-row seed counts (spans of row
//   k_scan_rows   slots summed, then scanned from the spans before them)
//   k_seed_write  per row slot: ordered compaction of chain starts (the
//                 tracklet id is the start cluster's index, so seeds come out
//                 sorted)
//   k_construct   one lane per tracklet: FP32 Kalman filter in registers,
//                 exact helix steps row by row, grid search with a chi^2 gate;
//                 all phases in one loop; tracklets of a sector group stay
//                 on one XCD
//   k_own         per sector chunk, in LDS: weight, 64-bit atomicMax owner key
//                 per cluster (order-free, smaller id wins ties), owned
//                 clusters per tracklet
//   k_tl_reduce,  >= min_clusters cut; track index and cluster offset of kept
//   k_tl_scan     tracklets (reduce spans of tracklets, then scan them with
//                 the span offsets)
//   k_output      one lane per tracklet: tracks, cluster lists, cluster->track
//
// No step depends on the order in which lanes or blocks run: every choice is
// the minimum of (value, index) and every list is built by prefix sums.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "tpc_internal.h"
#include "tpc_model.h"

namespace tpc {

constexpr int kGridBlock = 256;
constexpr int kMaxBins = 4096;   // bins per row (LDS counting sort)
constexpr int kGridWaveBins = 1024;  // LDS bins of the one-wave form of k_grid
// k_nf stages neighbour rows of up to CAP clusters in LDS and keeps up to
// LIST window candidates per row and lane: (512, 12) with 16-bit entries and
// four waves for rows of central density (31 KB of LDS, five workgroups per
// CU), (1024, 32) with 8-bit entries and eight waves for dense events (74 KB,
// two workgroups per CU: a dense row's clusters are shared by more waves),
// and (256, 12) with one wave for sparse rows (11 KB, fourteen workgroups per
// CU: many small events batched).  A lane's longer
// list is searched by its whole wave, a longer row by the global-memory
// search; every configuration gives the same links.
constexpr int kNfCapSmall = 512, kNfListSmall = 12;
constexpr int kNfCapLarge = 1024, kNfListLarge = 32;
constexpr int kNfCapWave = 256;
constexpr int kNfDenseBlock = 512;  // threads of the dense form's workgroups
constexpr int kScanBlock = 1024;
constexpr int kRowSpan = 8 * kScanBlock;  // row slots per workgroup of the row scan
constexpr int kTlBlock = 64;     // one wave per block for per-tracklet kernels

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Window test |a - b| <= w of the neighbours finder, decided in FP64: the
// difference of two FP32 values is then (for coordinates of this size) exact,
// so the decision is that of the exact values, and it is the same operation
// as the FP64 reference takes on the same FP32 inputs.  Three instructions,
// no branch.
__device__ __forceinline__ bool within(float a, float b, float w) {
  return fabs((double)a - (double)b) <= (double)w;
}
// Both coordinates of p inside the window around (yc, zc); both tests are
// always evaluated (no short-circuit branch).
__device__ __forceinline__ bool in_window(float2 p, float yc, float zc, float wy, float wz) {
  return ((int)within(p.x, yc, wy) & (int)within(p.y, zc, wz)) != 0;
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

// Counting sort of a row's clusters into its bins, counts in cnt[0..nb):
// LDS, or for a row with more bins than the LDS array holds global memory,
// read past the CU's cache and fenced before each barrier so that every
// lane sees the others' atomics.
template <int BS, bool G>
__device__ __forceinline__ void grid_sort(const DevEvent& ev, const Scratch& sc, const RowGrid& g,
                                          int b, int e, int nb, int* cnt, int* s_w) {
  const int tid = threadIdx.x, ny = g.ny;
  auto ld = [](int* p) {
    if constexpr (G) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  };
  auto sync = []() {
    if constexpr (G) __threadfence();
    __syncthreads();
  };
  for (int k = tid; k < nb; k += BS) cnt[k] = 0;
  sync();
  for (int i = b + tid; i < e; i += BS) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) continue;
    atomicAdd(&cnt[bin_z(g, z) * ny + bin_y(g, y)], 1);
  }
  sync();
  int tot;
  {  // exclusive scan of cnt[0..nb) in place, each thread a contiguous piece
    const int per = (nb + BS - 1) / BS;
    const int lo = tid * per, hi = min(lo + per, nb);
    int sum = 0;
    for (int k = lo; k < hi; ++k) sum += ld(&cnt[k]);
    int off = block_excl_scan<BS>(sum, s_w, &tot);
    for (int k = lo; k < hi; ++k) {
      int v = ld(&cnt[k]);
      cnt[k] = off;
      off += v;
    }
    sync();
  }
  for (int k = tid; k < nb; k += BS) sc.bins[g.bin_base + k] = ld(&cnt[k]);
  if (tid == 0) sc.bins[g.bin_base + nb] = tot;
  sync();
  for (int i = b + tid; i < e; i += BS) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) continue;
    int pos = atomicAdd(&cnt[bin_z(g, z) * ny + bin_y(g, y)], 1);
    GridRec rec;
    rec.y = y;
    rec.z = z;
    rec.id = i;
    rec.pad = 0;
    sc.g_rec[b + pos] = rec;
  }
}

// One workgroup of BS threads per row slot: the row's z range, its grid and
// the counting sort.  With BS = 64 (many sparse rows) the LDS counts hold
// NB bins; a row with more takes its counts in global memory, in the
// cluster links of its own clusters (up[b..e), written later by k_nf).
template <int BS, int NB>
__global__ __launch_bounds__(BS) void k_grid(DevEvent ev, KParams kp, Scratch sc,
                                             int32_t* cluster_track) {
  __shared__ int s_cnt[NB + 1];
  __shared__ float s_red[2][BS / 64];
  __shared__ int s_w[BS / 64];
  const int rs = blockIdx.x;
  const int R = ev.n_sectors * kp.n_rows;
  const int N = ev.n_dev ? *ev.n_dev : ev.n_clusters;
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
  for (int i = b + tid; i < e; i += BS) {
    float y = ev.y[i], z = ev.z[i];
    if (!isfinite(y) || !isfinite(z)) {
      ++nonfin;
      continue;
    }
    zmin = fminf(zmin, z);
    zmax = fmaxf(zmax, z);
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
  for (int i = 1; i < BS / 64; ++i) {
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
  // a row owns n + 1 bin slots (bins[] is laid out per row at b + rs): never
  // more bins than clusters, whatever the occupancy asks for
  int nbt = (int)((float)n / kp.bin_occupancy);
  nbt = min(nbt, min(n, kMaxBins));
  nbt = nbt < 1 ? 1 : nbt;
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
  if (nb <= NB)
    grid_sort<BS, false>(ev, sc, g, b, e, nb, s_cnt, s_w);
  else
    grid_sort<BS, true>(ev, sc, g, b, e, nb, sc.up + b, s_w);
}

// ------------------------------------------------------------------ k_nf

// The straightness of a candidate pair (section 1): d on row k-1, u on row
// k+1 and the cluster c of row k between them.  (ry, rz) = (1 - t)(d - c) +
// t (u - c) is how far the straight line through d and u passes from c on
// row k, with t = (x_k - x_{k-1}) / (x_{k+1} - x_{k-1}); chi^2 = (ry^2 /
// sigma_y^2 + rz^2 / sigma_z^2) / (1 + t^2 + (1 - t)^2).  a = (1 - t)(d - c)
// is taken once per d, and w = the inverse variances over the norm once per
// row.  Every search below evaluates chi^2 with these two functions, so the
// staged, the wave-wide and the global-memory searches give the same links.
struct NfMetric {
  float t, omt, wy, wz;
};
__device__ __forceinline__ float2 nf_a(const NfMetric& k, float2 d, float2 c) {
  return make_float2(k.omt * (d.x - c.x), k.omt * (d.y - c.y));
}
__device__ __forceinline__ float nf_chi2(const NfMetric& k, float2 a, float2 u, float2 c) {
  const float ry = fmaf(k.t, u.x - c.x, a.x), rz = fmaf(k.t, u.y - c.y, a.y);
  return fmaf(ry, ry * k.wy, rz * (rz * k.wz));
}

// Neighbour-row view staged in LDS.
struct RowView {
  const float2* yz;
  const uint16_t* id;    // cluster index - base
  const uint16_t* bins;  // bins of the row, index 0 = first bin
  RowGrid g;
  int base;
  __device__ float2 yz_at(int j) const { return yz[j]; }
  __device__ int id_at(int j) const { return base + id[j]; }
};

__device__ __forceinline__ float2 yz_off(const float2* yz, int off) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(yz) + off);
}

// Neighbour-row view in global memory (rows too large for the LDS stage).
struct RowViewG {
  const GridRec* rec;
  const int32_t* bins;
  RowGrid g;
  __device__ float2 yz_at(int j) const {
    const GridRec v = rec[j];
    return make_float2(v.y, v.z);
  }
  __device__ int id_at(int j) const { return rec[j].id; }
};


// Best (chi2, d, u) pair for a cluster at c of row k (section 1): every pair
// of window candidates, no lists (used for rows beyond the LDS stage).
template <class V>
__device__ __forceinline__ void nf_search(const V& D, const V& U, float2 c, const NfMetric& km,
                                          float wy, float wz, float& best, int& bd, int& bu) {
  const float m = 1e-3f;  // bin ranges are only an accelerator: widen them
  const int dy0 = bin_y(D.g, c.x - wy - m), dy1 = bin_y(D.g, c.x + wy + m);
  const int dz0 = bin_z(D.g, c.y - wz - m), dz1 = bin_z(D.g, c.y + wz + m);
  const int uy0 = bin_y(U.g, c.x - wy - m), uy1 = bin_y(U.g, c.x + wy + m);
  const int uz0 = bin_z(U.g, c.y - wz - m), uz1 = bin_z(U.g, c.y + wz + m);
  for (int iz = dz0; iz <= dz1; ++iz) {
    const int j0 = D.bins[iz * D.g.ny + dy0], j1 = D.bins[iz * D.g.ny + dy1 + 1];
    for (int j = j0; j < j1; ++j) {
      const float2 pd = D.yz_at(j);
      if (!in_window(pd, c.x, c.y, wy, wz)) continue;
      const int idd = D.id_at(j);
      const float2 a = nf_a(km, pd, c);
      for (int kz = uz0; kz <= uz1; ++kz) {
        const int k0 = U.bins[kz * U.g.ny + uy0], k1 = U.bins[kz * U.g.ny + uy1 + 1];
        for (int k = k0; k < k1; ++k) {
          const float2 pu = U.yz_at(k);
          if (!in_window(pu, c.x, c.y, wy, wz)) continue;
          const int idu = U.id_at(k);
          const float chi2 = nf_chi2(km, a, pu, c);
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

// Entries of a lane's candidate list.  uint16_t: the byte offset of the
// record in the LDS stage (8 x its position), used as it is.  uint8_t: the
// position relative to the lane's first candidate, so that twice as many
// entries fit the same LDS; a candidate more than 255 positions after the
// first does not fit.
template <class E>
struct NfEntry;
template <>
struct NfEntry<uint16_t> {
  __device__ static uint16_t enc(int j, int) { return (uint16_t)(j << 3); }
  __device__ static int off(int v, int) { return v; }
};
template <>
struct NfEntry<uint8_t> {
  __device__ static uint8_t enc(int j, int first) { return (uint8_t)(j - first); }
  __device__ static int off(int v, int first) { return (first + v) << 3; }
};

// Window candidates of one neighbour row, listed in column `lane` of a
// [LIST][blockDim] LDS array (NfEntry; *first = the first candidate's
// position).  Returns the count, or LIST + 1 if the list cannot hold them
// all.
template <int LIST, class E, int BS>
__device__ __forceinline__ int nf_collect(const RowView& V, float yc, float zc, float wy, float wz,
                                          E (*list)[BS], int lane, int* first) {
  const float m = 1e-3f;
  const int y0 = bin_y(V.g, yc - wy - m), y1 = bin_y(V.g, yc + wy + m);
  const int z0 = bin_z(V.g, zc - wz - m), z1 = bin_z(V.g, zc + wz + m);
  int cnt = 0, j0 = 0;
  bool far = false;
  // candidates come in position order (bin rows, then bins, of the grid)
  auto take = [&](int j, float2 p) {
    if (in_window(p, yc, zc, wy, wz)) {
      j0 = cnt ? j0 : j;
      if constexpr (sizeof(E) == 1) far |= j - j0 >= 256;
      if (cnt < LIST && !far) list[cnt][lane] = NfEntry<E>::enc(j, j0);
      ++cnt;
    }
  };
  // two bin rows' ranges are read together and the records four at a time,
  // so that one wait covers several LDS reads; the list keeps bin order
  for (int iz = z0; iz <= z1; iz += 2) {
    const int ib = min(iz + 1, z1) * V.g.ny;
    const int a0 = V.bins[iz * V.g.ny + y0], a1 = V.bins[iz * V.g.ny + y1 + 1];
    const int b0 = V.bins[ib + y0], b1 = V.bins[ib + y1 + 1];
    const int na = a1 - a0, n = na + (iz + 1 <= z1 ? b1 - b0 : 0);
    for (int k = 0; k < n; k += 4) {
      int j[4];
      float2 p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = min(k + u, n - 1);
        j[u] = kk < na ? a0 + kk : b0 + (kk - na);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = V.yz[j[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k + u < n) take(j[u], p[u]);
    }
  }
  *first = j0;
  return far ? LIST + 1 : cnt;
}

// Pair bookkeeping of one wave: its clusters' first pair, candidate counts
// in the upper row, coordinates, best pair keys and, for relative list
// entries, the first candidates' positions in both rows.
template <class E>
struct NfPairs {
  int off[64];
  uint16_t nu[64];
  float2 c[64];
  unsigned long long key[64];
  uint16_t first[2][sizeof(E) == 1 ? 64 : 1];
};

// LDS written by other lanes of the wave is visible after this.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Entry e of a wave's shared list: the 16-bit byte offset of a record in
// the stage, in the wave's columns of a list, 32 sizeof(E) entries a row.
template <class E, int BS>
__device__ __forceinline__ uint16_t& wave_slot(E (*list)[BS], int col0, int e) {
  constexpr int per = 32 * sizeof(E);
  return *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(&list[e / per][col0]) +
                                      2 * (e % per));
}

// Window candidates of one neighbour row for ONE cluster (yc, zc the same in
// every lane), listed by the whole wave into its columns of list (wave_slot),
// in bin order.  Returns the count (the list is incomplete beyond cap
// entries).
template <class E, int BS>
__device__ __forceinline__ int nf_wave_collect(const RowView& V, float yc, float zc, float wy,
                                               float wz, E (*list)[BS], int cap,
                                               int col0, int lane) {
  const float m = 1e-3f;
  const int y0 = bin_y(V.g, yc - wy - m), y1 = bin_y(V.g, yc + wy + m);
  const int z0 = bin_z(V.g, zc - wz - m), z1 = bin_z(V.g, zc + wz + m);
  int cnt = 0;
  for (int iz = z0; iz <= z1; ++iz) {
    const int j0 = V.bins[iz * V.g.ny + y0], j1 = V.bins[iz * V.g.ny + y1 + 1];
    for (int jb = j0; jb < j1; jb += 64) {
      const int j = jb + lane;
      const bool in = j < j1 && in_window(V.yz[min(j, j1 - 1)], yc, zc, wy, wz);
      const unsigned long long bal = __ballot(in);
      const int pos = cnt + __popcll(bal & ((1ull << lane) - 1ull));
      if (in && pos < cap) wave_slot(list, col0, pos) = (uint16_t)(j << 3);
      cnt += __popcll(bal);
    }
  }
  return cnt;
}

// The best pair key (chi^2 bits, d, u row-local indices; ~0 if none) of ONE
// cluster at c, searched by the whole wave: both candidate lists, then the
// pairs dealt out over the lanes and a 64-bit minimum.  *fits is false if a
// list exceeded cap (the key is then not valid).
template <class E, int BS>
__device__ __forceinline__ unsigned long long nf_wave_pairs(
    const RowView& D, const RowView& U, float2 c, const NfMetric& km, float wy, float wz,
    E (*s_dl)[BS], E (*s_ul)[BS], int cap, int col0, int lane, bool* fits) {
  const int nd = nf_wave_collect(D, c.x, c.y, wy, wz, s_dl, cap, col0, lane);
  const int nu = nd ? nf_wave_collect(U, c.x, c.y, wy, wz, s_ul, cap, col0, lane) : 0;
  *fits = nd <= cap && nu <= cap;
  unsigned long long best = ~0ull;
  if (!*fits || nu == 0) return best;
  wave_lds_sync();
  const int np = nd * nu, dp = 64 / nu, dq = 64 - dp * nu;
  int p = lane / nu, q = lane - (lane / nu) * nu;
  for (int k = lane; k < np; k += 64) {
    const int jd = wave_slot(s_dl, col0, p), ju = wave_slot(s_ul, col0, q);
    const float chi2 = nf_chi2(km, nf_a(km, yz_off(D.yz, jd), c), yz_off(U.yz, ju), c);
    const unsigned long long hi = (unsigned long long)__float_as_uint(chi2) << 32;
    if (hi <= best)
      best = min(best, hi | ((unsigned long long)D.id[jd >> 3] << 16) | (unsigned)U.id[ju >> 3]);
    q += dq;
    p += dp;
    if (q >= nu) {
      q -= nu;
      ++p;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) best = min(best, __shfl_xor(best, d, 64));
  return best;
}

// The staged neighbour search of a row's clusters (section 1), one cluster
// per lane.  Each lane lists its window candidates in both neighbour rows;
// then the pairs of the wave's 64 clusters are dealt out evenly (each lane
// walks a contiguous run of them, up to four pairs of one (cluster, d) at a
// time), so that a dense cluster does not hold up its wave.  The best pair of
// a cluster is the smallest (chi^2, d, u), with d and u the clusters' indices
// relative to their rows' first (16 bits each), whichever lane evaluated it:
// one 64-bit minimum per cluster in LDS.  Within a run a lane keeps only the
// smallest chi^2 and where it was found; an exact tie of chi^2 (rare) is
// decided on the indices on a separate path.  A cluster with more than LIST
// candidates in a row is searched by the whole wave afterwards
// (nf_wave_pairs).  The four reads of a group may run past the end of a
// u list, into rows cleared before the first round or left by an earlier
// one: s_ul has three rows more than LIST, and with relative entries the
// upper row's stage 256 records more than CAP, so that these reads stay in
// place; their pairs are not counted.
template <int CAP, int LIST, class E, int BS>
__device__ __forceinline__ void nf_pairs_staged(
    const DevEvent& ev, const KParams& kp, const Scratch& sc, int b, int e, int bd_, int bu_,
    const RowGrid& gd, const RowGrid& gu, const GridRec& me_first, const NfMetric& km,
    float wy, float wz, const float2* s_yzd, const float2* s_yzu, uint16_t (*s_id)[CAP],
    uint16_t (*s_bins)[CAP + 2], E (*s_dl)[BS], E (*s_ul)[BS], NfPairs<E>* s_pw) {
  constexpr bool kRel = sizeof(E) == 1;  // relative (8-bit) list entries
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, col0 = tid - lane;
  NfPairs<E>& P = s_pw[w];
  const RowView D{s_yzd, s_id[0], s_bins[0], gd, bd_}, U{s_yzu, s_id[1], s_bins[1], gu, bu_};
  const bool both = gd.n > 0 && gu.n > 0;
  for (int base = col0; base < e - b; base += BS) {  // uniform over the wave
    const int ii = base + lane;
    const bool have = ii < e - b;
    GridRec me = {};
    if (have) me = ii == tid ? me_first : sc.g_rec[b + ii];
    const float yc = me.y, zc = me.z;
    int nd = 0, nu = 0, fd = 0, fu = 0;
    if (have && both) {
      nd = nf_collect<LIST>(D, yc, zc, wy, wz, s_dl, tid, &fd);
      nu = nd ? nf_collect<LIST>(U, yc, zc, wy, wz, s_ul, tid, &fu) : 0;
    }
    const bool listed = nd <= LIST && nu <= LIST;
    const int np = listed ? nd * nu : 0;
    int incl = np;  // inclusive scan over the wave
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    P.off[lane] = incl - np;
    P.nu[lane] = nu;
    if constexpr (kRel) {
      P.first[0][lane] = fd;
      P.first[1][lane] = fu;
    }
    P.c[lane] = make_float2(yc, zc);
    P.key[lane] = ~0ull;
    wave_lds_sync();
    // this lane's run [k, kend) of the wave's pairs
    const int per = (total + 63) >> 6;
    int k = min(lane * per, total);
    const int kend = min(k + per, total);
    if (k < kend) {
      int o = 0;  // owner: the last cluster whose first pair is <= k
      for (int step = 32; step >= 1; step >>= 1)
        if (o + step < 64 && P.off[o + step] <= k) o += step;
      int nu_o = P.nu[o], db = 0, ub = 0;
      if constexpr (kRel) {
        db = P.first[0][o];
        ub = P.first[1][o];
      }
      int next = o < 63 ? P.off[o + 1] : total;
      float2 c = P.c[o];
      const int rel = k - P.off[o];
      int p = rel / nu_o, q = rel - p * nu_o;
      int jd = NfEntry<E>::off(s_dl[p][col0 + o], db);  // byte offsets into the stage
      float2 a = nf_a(km, yz_off(s_yzd, jd), c);
      float bc = INFINITY;  // the run's best for cluster o: chi^2, d and u offsets
      int bj = -1, bk = -1;
      auto flush = [&]() {
        if (bj >= 0)
          atomicMin(&P.key[o], ((unsigned long long)__float_as_uint(bc) << 32) |
                                   ((unsigned long long)s_id[0][bj >> 3] << 16) |
                                   (unsigned)s_id[1][bk >> 3]);
      };
      while (true) {
        // up to four pairs of the same (cluster, d) at once: their LDS reads
        // overlap
        const int m = min(4, min(nu_o - q, kend - k));
        const E* lu = &s_ul[q][col0 + o];
        int ku[4];
        float x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ku[i] = NfEntry<E>::off(lu[i * BS], ub);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = nf_chi2(km, a, yz_off(s_yzu, ku[i]), c);
        const float bc0 = bc;
        const int bj0 = bj, bk0 = bk;
        bool tie = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool v = i < m;
          tie |= v && x[i] == bc;
          const bool lt = v && x[i] < bc;
          bc = lt ? x[i] : bc;
          bj = lt ? jd : bj;
          bk = lt ? ku[i] : bk;
        }
        if (tie) {  // an exact tie of chi^2: the group again, on the full keys
          bc = bc0;
          bj = bj0;
          bk = bk0;
          for (int i = 0; i < m; ++i) {
            bool take = bj < 0 || x[i] < bc;
            if (!take && x[i] == bc) {
              const int d1 = s_id[0][jd >> 3], d0 = s_id[0][bj >> 3];
              take = d1 < d0 || (d1 == d0 && s_id[1][ku[i] >> 3] < s_id[1][bk >> 3]);
            }
            if (take) {
              bc = x[i];
              bj = jd;
              bk = ku[i];
            }
          }
        }
        k += m;
        q += m - 1;
        if (k == kend) break;
        if (k == next) {  // the next cluster with pairs
          flush();
          bc = INFINITY;
          bj = bk = -1;
          do {
            ++o;
          } while (o < 63 && P.off[o + 1] <= k);
          nu_o = P.nu[o];
          if constexpr (kRel) {
            db = P.first[0][o];
            ub = P.first[1][o];
          }
          next = o < 63 ? P.off[o + 1] : total;
          c = P.c[o];
          p = q = 0;
        } else if (++q == nu_o) {
          q = 0;
          ++p;
        } else {
          continue;
        }
        jd = NfEntry<E>::off(s_dl[p][col0 + o], db);
        a = nf_a(km, yz_off(s_yzd, jd), c);
      }
      flush();
    }
    wave_lds_sync();
    unsigned long long key = P.key[lane];
    bool alone = false;
    // a cluster with more than LIST candidates in a row: the wave takes each
    // in turn, listing its candidates in the wave's columns of the lists
    // (free now) and sharing its pairs
    for (unsigned long long ov = __ballot(!listed); ov; ov &= ov - 1ull) {
      const int o = __ffsll((unsigned long long)ov) - 1;
      bool fits;
      const unsigned long long ko =
          nf_wave_pairs(D, U, P.c[o], km, wy, wz, s_dl, s_ul, LIST * 32 * (int)sizeof(E), col0,
                        lane, &fits);
      if (lane == o) {
        key = ko;
        alone = !fits;
      }
      wave_lds_sync();  // the lists are rewritten for the next one
    }
    float best = INFINITY;
    int bd = -1, bu = -1;
    if (alone) {  // even the wave's lists overflow: nested bin scans
      nf_search(D, U, make_float2(yc, zc), km, wy, wz, best, bd, bu);
    } else if (key != ~0ull) {
      best = __uint_as_float((unsigned)(key >> 32));
      bd = bd_ + (int)((key >> 16) & 0xffffu);
      bu = bu_ + (int)(key & 0xffffu);
    }
    if (have) {
      const bool ok = bd >= 0 && best <= kp.nf_chi2_max;
      sc.up[me.id] = ok ? bu : -1;
      sc.dn[me.id] = ok ? bd : -1;
    }
    wave_lds_sync();  // P is rewritten by the next round
  }
}

template <int CAP, int LIST, class E, int BS>
__global__ __launch_bounds__(BS) void k_nf(DevEvent ev, KParams kp, Scratch sc) {
  static_assert(CAP * 8 <= 65536, "stage offsets are 16-bit");
  static_assert(LIST * 32 * (int)sizeof(E) >= CAP, "a wave's lists hold a whole staged row");
  __shared__ float2 s_yzd[CAP], s_yzu[CAP + (sizeof(E) == 1 ? 256 : 0)];
  __shared__ uint16_t s_id[2][CAP];
  __shared__ uint16_t s_bins[2][CAP + 2];
  __shared__ E s_dl[LIST][BS];
  __shared__ E s_ul[LIST + 3][BS];
  __shared__ NfPairs<E> s_pw[BS / 64];
  if (event_bad(sc.counters)) return;
  // blocks in row-major order over the sectors: the dense inner rows of every
  // sector start first, and the sparse outer rows fill in behind them
  const int r = blockIdx.x / ev.n_sectors;
  const int rs = (blockIdx.x - r * ev.n_sectors) * kp.n_rows + r;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  if (r == 0 || r == kp.n_rows - 1) {
    for (int i = b + tid; i < e; i += BS) {
      sc.up[i] = -1;
      sc.dn[i] = -1;
    }
    return;
  }
  // the thread's first cluster record, loaded together with the neighbour
  // rows' headers: it is needed only after the staging, and one level of
  // global-load latency fewer is on the workgroup's path
  GridRec me_first = {};
  if (tid < e - b) me_first = sc.g_rec[b + tid];
  const RowGrid gd = sc.grid[rs - 1], gu = sc.grid[rs + 1];
  const int bd_ = ev.ro[rs - 1], bu_ = ev.ro[rs + 1];
  // staged: both rows fit the LDS stage
  const bool stage = gd.n <= CAP && gu.n <= CAP;
  const float xd = kp.row_x[r - 1], xc = kp.row_x[r], xu = kp.row_x[r + 1];
  NfMetric km;
  km.t = (xc - xd) / (xu - xd);
  km.omt = 1.f - km.t;
  const float inorm = 1.f / (1.f + km.t * km.t + km.omt * km.omt);
  km.wy = inorm / kp.sy2;
  km.wz = inorm / kp.sz2;
  const float wy = kp.nf_win_y, wz = kp.nf_win_z;
  if (stage) {
    const int nbd = gd.ny * gd.nz, nbu = gu.ny * gu.nz;
    for (int i = tid; i < gd.n; i += BS) {
      const GridRec v = sc.g_rec[bd_ + i];
      s_yzd[i] = make_float2(v.y, v.z);
      s_id[0][i] = (uint16_t)(v.id - bd_);
    }
    for (int i = tid; i < gu.n; i += BS) {
      const GridRec v = sc.g_rec[bu_ + i];
      s_yzu[i] = make_float2(v.y, v.z);
      s_id[1][i] = (uint16_t)(v.id - bu_);
    }
    if (gd.n > 0)
      for (int i = tid; i <= nbd; i += BS) s_bins[0][i] = (uint16_t)sc.bins[gd.bin_base + i];
    if (gu.n > 0)
      for (int i = tid; i <= nbu; i += BS) s_bins[1][i] = (uint16_t)sc.bins[gu.bin_base + i];
    for (int i = 0; i < LIST + 3; ++i) s_ul[i][tid] = 0;
    __syncthreads();
  }
  // lanes take the row's clusters in grid order: neighbouring lanes sit at
  // nearby positions and visit similar bins, so a wave diverges less
  if (stage) {
    nf_pairs_staged<CAP, LIST, E, BS>(ev, kp, sc, b, e, bd_, bu_, gd, gu, me_first, km, wy, wz, s_yzd,
                               s_yzu, s_id, s_bins, s_dl, s_ul, s_pw);
    return;
  }
  for (int ii = tid; ii < e - b; ii += BS) {
    const GridRec me = ii == tid ? me_first : sc.g_rec[b + ii];
    const int i = me.id;
    float best = INFINITY;
    int bd = -1, bu = -1;
    if (gd.n > 0 && gu.n > 0) {
      const RowViewG D{sc.g_rec + bd_, sc.bins + gd.bin_base, gd};
      const RowViewG U{sc.g_rec + bu_, sc.bins + gu.bin_base, gu};
      nf_search(D, U, make_float2(me.y, me.z), km, wy, wz, best, bd, bu);
    }
    const bool ok = bd >= 0 && best <= kp.nf_chi2_max;
    sc.up[i] = ok ? bu : -1;
    sc.dn[i] = ok ? bd : -1;
  }
}

// ------------------------------------------------------------------ k_evo

template <int BS>
__global__ __launch_bounds__(BS) void k_evo(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ int s_w[BS / 64];
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  int cnt = 0;
  for (int i = b + tid; i < e; i += BS) {
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
  block_excl_scan<BS>(cnt, s_w, &tot);
  if (tid == 0) sc.row_cnt[rs] = tot;
}

// ------------------------------------------------------------------ scans

// The per-row seed counts are scanned in spans of kRowSpan row slots, one
// workgroup each (a batch of many events has hundreds of thousands of row
// slots): k_rows_reduce sums every span, k_scan_rows scans each span from
// the sum of the spans before it.  A span goes through LDS, so that global
// reads and writes are coalesced while every thread scans eight consecutive
// slots.
__global__ __launch_bounds__(kScanBlock) void k_rows_reduce(int R, Scratch sc) {
  __shared__ int s_w[kScanBlock / 64];
  if (event_bad(sc.counters)) return;
  const int base = blockIdx.x * kRowSpan;
  int sum = 0;
#pragma unroll
  for (int q = 0; q < kRowSpan / kScanBlock; ++q) {
    const int i = base + q * kScanBlock + (int)threadIdx.x;
    sum += i < R ? sc.row_cnt[i] : 0;
  }
  int tot;
  block_excl_scan<kScanBlock>(sum, s_w, &tot);
  if (threadIdx.x == 0) sc.row_part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_rows(int R, Scratch sc) {
  __shared__ int s_w[kScanBlock / 64];
  __shared__ int s_v[kRowSpan + kRowSpan / 32];  // one pad word per 32
  if (event_bad(sc.counters)) return;
  constexpr int kPer = kRowSpan / kScanBlock;
  const int tid = threadIdx.x, base = blockIdx.x * kRowSpan;
  auto at = [](int k) { return k + (k >> 5); };
  // offset of this span: the sums of the spans before it
  int pre = 0;
  for (int j = tid; j < (int)blockIdx.x; j += kScanBlock) pre += sc.row_part[j];
  int off;
  block_excl_scan<kScanBlock>(pre, s_w, &off);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int k = q * kScanBlock + tid;
    s_v[at(k)] = base + k < R ? sc.row_cnt[base + k] : 0;
  }
  __syncthreads();
  int v[kPer], sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = s_v[at(tid * kPer + q)];
    sum += v[q];
  }
  int tot;
  int run = off + block_excl_scan<kScanBlock>(sum, s_w, &tot);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    s_v[at(tid * kPer + q)] = run;
    run += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int k = q * kScanBlock + tid;
    if (base + k < R) sc.row_cnt[base + k] = s_v[at(k)];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 0) {
    const int all = off + tot;
    sc.row_cnt[R] = all;
    sc.counters[C_SEEDS] = all;
    if (all > sc.cap_tl) atomicOr(&sc.counters[C_ERR], E_TL_OVERFLOW);
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_seed_write(DevEvent ev, Scratch sc) {
  __shared__ int s_w[BS / 64];
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int tid = threadIdx.x;
  const int b = ev.ro[rs], e = ev.ro[rs + 1];
  int base = sc.row_cnt[rs];
  if (sc.row_cnt[rs + 1] == base) return;  // uniform: no start in this row
  for (int c0 = b; c0 < e; c0 += BS) {
    const int i = c0 + tid;
    const int f = (i < e) ? sc.start[i] : 0;
    int tot;
    const int rank = block_excl_scan<BS>(f, s_w, &tot);
    if (f && base + rank < sc.cap_tl) {
      sc.seeds[base + rank] = i;
      sc.seed_rs[base + rank] = rs;
    }
    base += tot;
  }
}

// ------------------------------------------------------------------ track model
//
// propagate, kf_update, seed3, rotate and step_par are in tpc_model.h.

// Work done by one lane of the constructor (for the algorithmic FLOP count).
struct Work {
  int steps = 0, updates = 0, cands = 0;
};

struct AcceptAll {
  __device__ bool operator()(const GridRec&) const { return true; }
};

// Best cluster of a row inside the chi^2 gate (smallest (chi2, index)) among
// those `accept` admits; its coordinates come back with it, so no reload is
// needed.
template <class Accept = AcceptAll>
__device__ __forceinline__ int search_row(const Scratch& sc, const RowGrid& g, int rb,
                                          const KState& s, const KParams& kp, float& by,
                                          float& bz_, Work& wk, Accept accept = Accept()) {
  if (g.n == 0) return -1;
  const float S00 = (float)(s.C.c00 + kp.sy2), S01 = (float)s.C.c10,
              S11 = (float)(s.C.c11 + kp.sz2);
  const float idet = frcp(S00 * S11 - S01 * S01);
  const float wy = fsqrt(kp.chi2_gate * S00) * 1.001f + 1e-4f;
  const float wz = fsqrt(kp.chi2_gate * S11) * 1.001f + 1e-4f;
  const int iy0 = bin_y(g, s.y - wy), iy1 = bin_y(g, s.y + wy);
  const int iz0 = bin_z(g, s.z - wz), iz1 = bin_z(g, s.z + wz);
  float best = INFINITY;
  int bid = -1;
  // the best is the smallest (chi^2, id) inside the gate, whatever the order
  // of the candidates: two bin rows' ranges are loaded together and their
  // records eight at a time, so that one wait covers a whole window in most
  // searches
  auto consider = [&](const GridRec& v) {
    const float ry = v.y - s.y, rz = v.z - s.z;
    const float chi2 = (ry * ry * S11 - 2.f * ry * rz * S01 + rz * rz * S00) * idet;
    if (chi2 <= kp.chi2_gate && (chi2 < best || (chi2 == best && v.id < bid)) && accept(v)) {
      best = chi2;
      bid = v.id;
      by = v.y;
      bz_ = v.z;
    }
  };
  for (int iz = iz0; iz <= iz1; iz += 2) {
    const int ia = g.bin_base + iz * g.ny, ib = g.bin_base + min(iz + 1, iz1) * g.ny;
    const int a0 = sc.bins[ia + iy0], a1 = sc.bins[ia + iy1 + 1];
    const int b0 = sc.bins[ib + iy0], b1 = sc.bins[ib + iy1 + 1];
    const int na = a1 - a0, n = na + (iz + 1 <= iz1 ? b1 - b0 : 0);
    wk.cands += n;
    for (int k = 0; k < n; k += 8) {
      GridRec v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = min(k + u, n - 1);
        v[u] = sc.g_rec[rb + (kk < na ? a0 + kk : b0 + (kk - na))];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k + u < n) consider(v[u]);
    }
  }
  return bid;
}

// ------------------------------------------------------------------ k_construct
//
// One lane per tracklet.  A lane's construction is a single loop of row
// steps, whatever phase it is in, so that the lanes of a wave stay in step:
//   P_CHAIN  outward through the chain, clusters taken unconditionally
//   P_UP     outward extension: search the row, chi^2 gate
//   P_REFIT  inward from the outermost cluster with a fresh covariance
//   P_DOWN   inward extension below the innermost cluster
// Two schedules run the same lane steps and give bitwise the same tracklets:
//   k_construct_rows   row-synchronous: a one-wave workgroup takes up to 64
//                      tracklets of ONE sector and walks the rows outward,
//                      then inward, in lockstep; the row being searched is
//                      staged in LDS (the next one is loaded while the
//                      current one is used), so the search costs LDS reads
//                      instead of two dependent global loads per step
//   k_construct_lanes  each lane runs its own tracklet through all its steps
//                      and takes the next one from a queue

enum Phase { P_CHAIN = 0, P_UP = 1, P_REFIT = 2, P_DOWN = 3, P_DONE = 4 };

// End state of a tracklet (global tracking), kEndStride floats: x and the
// state (floats 0-5), the validity flag (float 6), then the packed FP64
// covariance from float 8 on; ten 16-byte stores.
constexpr int kEndValid = 6;
constexpr int kEndCov = 8;
__device__ __forceinline__ const double* end_cov(const float* E) {
  return reinterpret_cast<const double*>(E + kEndCov);
}
__device__ __forceinline__ void store_end(float* E, const KState& s) {
  float4* q = reinterpret_cast<float4*>(E);
  double2* w = reinterpret_cast<double2*>(E + kEndCov);
  const Cov& C = s.C;
  q[0] = make_float4(s.x, s.y, s.z, s.sp);
  q[1] = make_float4(s.tl, s.qpt, 0.f, 0.f);
  w[0] = make_double2(C.c00, C.c10);
  w[1] = make_double2(C.c11, C.c20);
  w[2] = make_double2(C.c21, C.c22);
  w[3] = make_double2(C.c30, C.c31);
  w[4] = make_double2(C.c32, C.c33);
  w[5] = make_double2(C.c40, C.c41);
  w[6] = make_double2(C.c42, C.c43);
  w[7] = make_double2(C.c44, 0.0);
}
__device__ __forceinline__ void load_end(const float* E, KState& s) {
  const float4* q = reinterpret_cast<const float4*>(E);
  const double2* w = reinterpret_cast<const double2*>(E + kEndCov);
  const float4 a = q[0], b = q[1];
  const double2 w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4], w5 = w[5], w6 = w[6],
                w7 = w[7];
  s.x = a.x; s.y = a.y; s.z = a.z; s.sp = a.w;
  s.tl = b.x; s.qpt = b.y;
  Cov& C = s.C;
  C.c00 = w0.x; C.c10 = w0.y; C.c11 = w1.x; C.c20 = w1.y; C.c21 = w2.x; C.c22 = w2.y;
  C.c30 = w3.x; C.c31 = w3.y; C.c32 = w4.x; C.c33 = w4.y;
  C.c40 = w5.x; C.c41 = w5.y; C.c42 = w6.x; C.c43 = w6.y;
  C.c44 = w7.x;
}

// ENDS: also record what global tracking starts from: the outward filter at
// the outermost collected cluster and the inward fit at the innermost one.
// Rows without a cluster do not update the state, so each is stored once,
// when its pass ends (the state then sits some miss rows beyond its cluster),
// and k_prolong carries it back to that cluster's row with one helix step.
// LDSH: the cluster of every row the tracklet visits is kept in the lane's
// row slots in LDS (H), and only the rows inner..outer go out to the hits
// array, once, at emit; the inward refit reads a row's coordinates through
// its cluster index.  Otherwise H is the tracklet's row of the hits array and
// the collected clusters' coordinates are stored beside it (HY), so that
// the refit reads them without a dependent load.  Both give the same
// tracklets.
template <bool ENDS, bool LDSH = false>
struct Lane {
  KState s;
  int t = 0, phase = P_DONE, r = 0, k0 = 0, rsb = 0, last_row = 0, misses = 0, n = 0, inner = 0;
  int cn = -1, cnn = -1;      // chain: cluster of row r and the one after
  float cy = 0.f, cz = 0.f;   // coordinates of cn / of the prefetched refit hit
  int hc = -1;                // refit: cluster of row r
  float l_sp = 0.f, l_tl = 0.f, l_q = 0.f, l_y = 0.f, l_z = 0.f;  // state at last hit
  float chi2 = 0.f;
  float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f, o4 = 0.f, o5 = 0.f;  // output state
  bool dropped = false;
  int32_t* H = nullptr;   // LDSH: this lane's kHitStride row slots in LDS
  float2* HY = nullptr;
  // the hit of the last step, stored at the start of the next one (or at the
  // end), so that no wait for loads of a step also waits for these stores
  int pend_r = -1, pend_h = -1;
  bool pend_yz = false;
  float pend_y = 0.f, pend_z = 0.f;

  __device__ void flush() {
    if (pend_r >= 0) {
      H[pend_r] = pend_h;
      if constexpr (!LDSH) {
        if (pend_yz) HY[pend_r] = make_float2(pend_y, pend_z);
      }
      pend_r = -1;
    }
  }

  __device__ bool outward() const { return phase == P_CHAIN || phase == P_UP; }
  __device__ bool inward() const { return phase == P_REFIT || phase == P_DOWN; }
  __device__ bool extending() const { return phase == P_UP || phase == P_DOWN; }

  // Set up tracklet tt: walk the seed window of its chain, fit the seed.
  __device__ void begin(int tt, const DevEvent& ev, const KParams& kp, const Scratch& sc,
                        const float* s_x) {
    const int nr = kp.n_rows;
    t = tt;
    const int start = sc.seeds[tt];
    const int rs0 = sc.seed_rs[tt];
    k0 = rs0 % nr;
    rsb = rs0 - k0;
    if constexpr (!LDSH) {
      H = sc.hits + (size_t)tt * kHitStride;
      HY = sc.hit_yz + (size_t)tt * kHitStride;
    }
    int m = 0, c = start, last = start, c1 = -1, c2 = -1;
    while (c >= 0 && m < kp.seed_window && k0 + m < nr) {
      H[k0 + m] = c;
      last = c;
      if (m == 1) c1 = c;
      if (m == 2) c2 = c;
      ++m;
      c = sc.up2[c];
    }
    if (m == 2) c2 = c;  // the chain may continue past a 2-cluster window
    const int bmid = H[k0 + m / 2];
    seed3(s, s_x[k0], ev.y[start], ev.z[start], s_x[k0 + m / 2], ev.y[bmid], s_x[k0 + m - 1],
          ev.y[last], ev.z[last], kp);
    dropped = fabsf(s.sp) > kp.max_sinphi;
    last_row = k0;
    l_sp = s.sp; l_tl = s.tl; l_q = s.qpt; l_y = s.y; l_z = s.z;
    if constexpr (!LDSH) HY[k0] = make_float2(s.y, s.z);
    phase = P_CHAIN;
    r = k0 + 1;
    cn = c1;
    cnn = c2;
    if (cn >= 0) {
      cy = ev.y[cn];
      cz = ev.z[cn];
    }
    misses = 0;
    n = 0;
    chi2 = 0.f;
  }

  // Inward refit set-up from the outermost collected cluster.
  __device__ void begin_refit(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                              const float* s_x) {
    if constexpr (ENDS) store_end(sc.ends + ((size_t)t * 2 + 1) * kEndStride, s);
    s.x = s_x[last_row];
    s.y = l_y;
    s.z = l_z;
    s.sp = l_sp;
    s.tl = l_tl;
    s.qpt = l_q;
    reset_cov(s.C, kp);
    n = 1;
    inner = last_row;
    chi2 = 0.f;
    o0 = s.x; o1 = s.y; o2 = s.z; o3 = s.sp; o4 = s.tl; o5 = s.qpt;
    phase = P_REFIT;
    r = last_row - 1;
    prefetch_refit(ev);
  }

  // Cluster of row r and its coordinates (used only if the row has a
  // cluster): without LDSH both loads are in flight at once.
  __device__ void prefetch_refit(const DevEvent& ev) {
    if (r >= k0) {
      hc = H[r];
      if constexpr (LDSH) {
        cy = ev.y[max(hc, 0)];
        cz = ev.z[max(hc, 0)];
      } else {
        const float2 v = HY[r];
        cy = v.x;
        cz = v.y;
      }
    }
  }

  // One row step at row r.  search(my, mz) returns the best cluster of the
  // row inside the chi^2 gate (or -1) and its coordinates.  Returns true when
  // the tracklet is finished (or dropped).
  template <class Search>
  __device__ bool step(const DevEvent& ev, const KParams& kp, const Scratch& sc, const float* s_x,
                       Search&& search, Work& wk) {
    const int nr = kp.n_rows;
    bool finish = false;
    const bool ext = extending();
    flush();
    // 0. the known measurement of the NEXT step (chain, refit) is loaded now,
    //    so that it has a whole step to arrive
    const bool pf_chain = phase == P_CHAIN && cnn >= 0 && r + 1 < nr;
    const bool pf_refit = phase == P_REFIT && r - 1 >= k0;
    float ny = 0.f, nz = 0.f;
    int nc = -1;
    if (pf_chain) {
      ny = ev.y[cnn];
      nz = ev.z[cnn];
      nc = sc.up2[cnn];
    } else if (pf_refit) {
      nc = H[r - 1];
      if constexpr (LDSH) {
        ny = ev.y[max(nc, 0)];
        nz = ev.z[max(nc, 0)];
      } else {
        const float2 v = HY[r - 1];
        ny = v.x;
        nz = v.y;
      }
    }
    // 1. one helix step for every lane, whatever its phase
    const bool ok = propagate(s, s_x[r], kp);
    if (ok) ++wk.steps;
    // 2. the measurement of this row: known (chain, refit) or searched
    int st = 2;  // 0 = cluster, 1 = no cluster (miss), 2 = stop
    int hit = -1;
    float my = cy, mz = cz;
    if (ok) {
      if (phase == P_CHAIN) {
        st = 0;
        hit = cn;
      } else if (phase == P_REFIT) {
        st = hc >= 0 ? 0 : 1;
        hit = hc;
      } else if (!(fabsf(s.z) > kp.z_max)) {
        st = 1;
        if (!(fabsf(s.y) > s_x[r] * kp.tan_half)) {
          hit = search(my, mz);
          if (hit >= 0) st = 0;
        }
      }
    }
    // 3. one Kalman update for every lane that has a cluster
    float c2 = 0.f;
    if (st == 0) {
      c2 = kf_update(s, my, mz, kp);
      ++wk.updates;
    }
    // 4. bookkeeping of the phase
    if (st == 2 && !ext) {
      dropped = finish = true;  // a step through known clusters failed
    } else if (phase == P_CHAIN || phase == P_UP) {
      if (st == 0) {
        last_row = r;
        l_sp = s.sp; l_tl = s.tl; l_q = s.qpt; l_y = my; l_z = mz;
      }
      if (st != 2) {  // H[r] = hit, HY[r] = (my, mz) if a cluster was taken
        pend_r = r;
        pend_h = hit;
        pend_yz = st == 0;
        pend_y = my;
        pend_z = mz;
      }
      if (phase == P_CHAIN) {
        cn = cnn;
        ++r;
        if (pf_chain) {  // cn >= 0 && r < nr
          cy = ny;
          cz = nz;
          cnn = nc;
        } else {
          phase = P_UP;
          misses = 0;
          if (r >= nr) begin_refit(ev, kp, sc, s_x);
        }
      } else {
        misses = st == 0 ? 0 : misses + 1;
        ++r;
        if (st == 2 || misses > kp.max_miss || r >= nr) begin_refit(ev, kp, sc, s_x);
      }
    } else {  // P_REFIT or P_DOWN: collected clusters enter the final fit
      if (st == 0) {
        chi2 += c2;
        ++n;
        inner = r;
        o0 = s.x; o1 = s.y; o2 = s.z; o3 = s.sp; o4 = s.tl; o5 = s.qpt;
      }
      if (phase == P_DOWN) {
        if (st != 2) {  // H[r] = hit
          pend_r = r;
          pend_h = hit;
          pend_yz = false;
        }
        misses = st == 0 ? 0 : misses + 1;
        --r;
        if (st == 2 || misses > kp.max_miss || r < 0) finish = true;
      } else {
        --r;
        if (pf_refit) {  // r >= k0
          hc = nc;
          cy = ny;
          cz = nz;
        }
      }
    }
    // a refit that reaches (or starts) below the chain start continues as P_DOWN
    if (!finish && phase == P_REFIT && r < k0) {
      phase = P_DOWN;
      misses = 0;
      if (r < 0) finish = true;
    }
    return finish;
  }

  // Tracklet outputs; the lane is done.
  __device__ void emit(const Scratch& sc) {
    flush();
    if constexpr (ENDS) {
      if (!dropped) store_end(sc.ends + (size_t)t * 2 * kEndStride, s);
    }
    if (dropped) {
      sc.row_lo[t] = 0;
      sc.row_hi[t] = -1;
      sc.n[t] = 0;
      sc.ndf[t] = 0;
      sc.chi2[t] = 0.f;
    } else {
      sc.row_lo[t] = inner;
      sc.row_hi[t] = last_row;
      sc.n[t] = n;
      sc.ndf[t] = 2 * n - 5;
      sc.chi2[t] = chi2;
      if constexpr (LDSH) {
        // rows inner..last_row out to the hits array, four at a time (the
        // other rows of the first and last four are never read)
        int4* G = reinterpret_cast<int4*>(sc.hits + (size_t)t * kHitStride);
        const int4* S = reinterpret_cast<const int4*>(H);
        for (int q = inner >> 2; q <= last_row >> 2; ++q) G[q] = S[q];
      }
    }
    sc.owned[t] = 0;  // summed over the sector's chunks by k_own
    float* P = sc.par + (size_t)t * 6;
    P[0] = dropped ? 0.f : o0; P[1] = dropped ? 0.f : o1; P[2] = dropped ? 0.f : o2;
    P[3] = dropped ? 0.f : o3; P[4] = dropped ? 0.f : o4; P[5] = dropped ? 0.f : o5;
    phase = P_DONE;
  }
};

// One atomic per wave and counter for the work done.
__device__ __forceinline__ void flush_work(const Work& wk, const Scratch& sc) {
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

// ---- row-synchronous schedule

constexpr int kRowLds = 1024;           // clusters of a row staged in LDS
constexpr int kStage = kRowLds / 64;    // staged records per lane
constexpr int kStageBins = kStage + 1;  // staged bin starts per lane (nb + 1 <= n + 1)

// A row of the search grid staged in LDS (row-local positions and bins).
struct RowStage {
  float2 yz[kRowLds];
  int32_t id[kRowLds];
  int32_t bins[kRowLds + 1];
};

// Next row held in registers between its loads (start of an iteration) and
// its LDS stores (end of the iteration), so the loads overlap the step.
struct StageRegs {
  GridRec rec[kStage];
  int32_t bin[kStageBins];
};

__device__ __forceinline__ bool stageable(const RowGrid& g) { return g.n <= kRowLds; }

__device__ __forceinline__ void stage_load(const Scratch& sc, const RowGrid& g, int row_first,
                                           StageRegs& R) {
  const int lane = threadIdx.x & 63;
  if (!stageable(g) || g.n == 0) return;
  const int nb = g.ny * g.nz;
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int j = k * 64 + lane;
    if (j < g.n) R.rec[k] = sc.g_rec[row_first + j];
  }
#pragma unroll
  for (int k = 0; k < kStageBins; ++k) {
    const int j = k * 64 + lane;
    if (j <= nb) R.bin[k] = sc.bins[g.bin_base + j];
  }
}

__device__ __forceinline__ void stage_store(const RowGrid& g, const StageRegs& R, RowStage& L) {
  const int lane = threadIdx.x & 63;
  if (!stageable(g) || g.n == 0) return;
  const int nb = g.ny * g.nz;
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int j = k * 64 + lane;
    if (j < g.n) {
      L.yz[j] = make_float2(R.rec[k].y, R.rec[k].z);
      L.id[j] = R.rec[k].id;
    }
  }
#pragma unroll
  for (int k = 0; k < kStageBins; ++k) {
    const int j = k * 64 + lane;
    if (j <= nb) L.bins[j] = R.bin[k];
  }
}

// search_row on a row staged in LDS: same candidates, same order, same
// arithmetic, so the same result.
__device__ __forceinline__ int search_row_lds(const RowStage& L, const RowGrid& g, const KState& s,
                                              const KParams& kp, float& by, float& bz_, Work& wk) {
  if (g.n == 0) return -1;
  const float S00 = (float)(s.C.c00 + kp.sy2), S01 = (float)s.C.c10,
              S11 = (float)(s.C.c11 + kp.sz2);
  const float idet = frcp(S00 * S11 - S01 * S01);
  const float wy = fsqrt(kp.chi2_gate * S00) * 1.001f + 1e-4f;
  const float wz = fsqrt(kp.chi2_gate * S11) * 1.001f + 1e-4f;
  const int iy0 = bin_y(g, s.y - wy), iy1 = bin_y(g, s.y + wy);
  const int iz0 = bin_z(g, s.z - wz), iz1 = bin_z(g, s.z + wz);
  float best = INFINITY;
  int bid = -1;
  for (int iz = iz0; iz <= iz1; ++iz) {
    const int j0 = L.bins[iz * g.ny + iy0];
    const int j1 = L.bins[iz * g.ny + iy1 + 1];
    wk.cands += j1 - j0;
    for (int j = j0; j < j1; ++j) {
      const float2 v = L.yz[j];
      const float ry = v.x - s.y, rz = v.y - s.z;
      const float chi2 = (ry * ry * S11 - 2.f * ry * rz * S01 + rz * rz * S00) * idet;
      if (chi2 <= kp.chi2_gate) {
        const int id = L.id[j];
        if (chi2 < best || (chi2 == best && id < bid)) {
          best = chi2;
          bid = id;
          by = v.x;
          bz_ = v.y;
        }
      }
    }
  }
  return bid;
}

// The row-synchronous workgroup is ONE wave: LDS operations of a wave are
// performed in order, so LDS written by its lanes is visible to its later
// reads without a workgroup barrier (whose memory fence would also wait for
// every global load and store in flight).  wave_sync only keeps the compiler
// from moving LDS accesses across it.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
// s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15): wait for vector memory only
constexpr int kWaitVm0 = 0x0F70;

template <bool ENDS>
__global__ __launch_bounds__(64) void k_construct_rows(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ float s_x[TPC_MAX_ROWS];
  __shared__ RowGrid s_hdr[TPC_MAX_ROWS];  // grid headers of the current sector's rows
  __shared__ RowStage s_row[2];
  if (event_bad(sc.counters)) return;
  const int lane = threadIdx.x;
  const int nr = kp.n_rows;
  for (int i = lane; i < nr; i += 64) s_x[i] = kp.row_x[i];
  wave_sync();
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  Work wk;

  // Work items are (sector, chunk of 64 tracklets).  Workgroups b = g (mod G)
  // take the chunks of the sectors s = g (mod G), G = min(8, sectors), in
  // order, with a stride of
  // the number of such workgroups: one XCD (one L2) stages the rows of only
  // a few sectors.  Any mapping gives the same results.
  const int G = min(8, ev.n_sectors);
  const int grp = blockIdx.x % G;
  const int nwg = ((int)gridDim.x - grp + G - 1) / G;
  for (int item = blockIdx.x / G;; item += nwg) {
    // find the sector of this item: prefix of chunk counts over the group
    int sec = -1, q = 0, base = 0;
    for (int s0 = grp; s0 < ev.n_sectors; s0 += G * 64) {
      const int sct = s0 + G * lane;
      int ch = 0;
      if (sct < ev.n_sectors) {
        const int a = min(sc.row_cnt[sct * nr], n_tl), b = min(sc.row_cnt[(sct + 1) * nr], n_tl);
        ch = (b - a + 63) >> 6;
      }
      const int inc = wave_incl_scan(ch);
      const int tot = __shfl(inc, 63, 64);
      if (item < base + tot) {
        const bool here = base + inc - ch <= item && item < base + inc;
        const unsigned long long m = __ballot(here);
        const int L = __ffsll((long long)m) - 1;
        sec = s0 + G * L;
        q = item - (base + __shfl(inc - ch, L, 64));
        break;
      }
      base += tot;
    }
    sec = __builtin_amdgcn_readfirstlane(sec);
    if (sec < 0) break;  // no more items for this workgroup
    q = __builtin_amdgcn_readfirstlane(q);
    const int rsb = sec * nr;
    wave_sync();  // the previous item's readers of s_hdr are done (in order)
    for (int i = lane; i < nr; i += 64) s_hdr[i] = sc.grid[rsb + i];
    const int tA = min(sc.row_cnt[rsb], n_tl), tB = min(sc.row_cnt[rsb + nr], n_tl);
    const int t = tA + q * 64 + lane;
    Lane<ENDS> ln;
    if (t < tB) {
      ln.begin(t, ev, kp, sc, s_x);
      if (ln.dropped) ln.emit(sc);
    }
    wave_sync();
    StageRegs R;
    // two passes over the rows: outward (dir +1), then inward (dir -1)
    for (int dir = 1; dir >= -1; dir -= 2) {
      const bool outw = dir > 0;
      auto active = [&]() { return outw ? ln.outward() : ln.inward(); };
      // first row of the pass: the smallest (outward) or largest (inward) pending row
      int ir = (ln.phase != P_DONE && active()) ? ln.r : (outw ? nr : -1);
      for (int d = 32; d >= 1; d >>= 1) {
        const int o = __shfl_xor(ir, d, 64);
        ir = outw ? min(ir, o) : max(ir, o);
      }
      ir = __builtin_amdgcn_readfirstlane(ir);
      if (ir < 0 || ir >= nr) continue;
      // pipeline: row ir in LDS buffer cur, row ir + dir in registers
      // (loaded one iteration ago), row ir + 2 dir loaded during this one
      int cur = 0;
      {
        const RowGrid g0 = s_hdr[ir];
        stage_load(sc, g0, g0.bin_base - (rsb + ir), R);
        stage_store(g0, R, s_row[cur]);
        const int i1 = ir + dir;
        if (i1 >= 0 && i1 < nr) {
          const RowGrid g1 = s_hdr[i1];
          stage_load(sc, g1, g1.bin_base - (rsb + i1), R);
        }
      }
      wave_sync();
      while (true) {
        const int i1 = ir + dir, i2 = ir + 2 * dir;
        const bool more = i1 >= 0 && i1 < nr;
        // everything issued in the previous iteration (a whole step ago) has
        // arrived: waiting here, once, keeps waits out of the step
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        if (more) {  // row ir + dir: registers -> the other buffer
          stage_store(s_hdr[i1], R, s_row[cur ^ 1]);
          if (i2 >= 0 && i2 < nr) {
            const RowGrid g2 = s_hdr[i2];
            stage_load(sc, g2, g2.bin_base - (rsb + i2), R);
          }
        }
        wave_sync();
        if (active() && ln.r == ir) {
          const RowGrid g = s_hdr[ir];
          const RowStage& L = s_row[cur];
          auto search = [&](float& my, float& mz) {
            if (stageable(g)) return search_row_lds(L, g, ln.s, kp, my, mz, wk);
            return search_row(sc, g, g.bin_base - (rsb + ir), ln.s, kp, my, mz, wk);
          };
          if (ln.step(ev, kp, sc, s_x, search, wk)) ln.emit(sc);
        }
        const bool go = __ballot(ln.phase != P_DONE && active()) != 0ull && more;
        if (!go) break;
        wave_sync();
        cur ^= 1;
        ir = i1;
      }
      wave_sync();  // the buffers are reused by the next pass
    }
  }
  flush_work(wk, sc);
}

// ---- lane schedule

template <bool ENDS, bool LDSH>
__global__ __launch_bounds__(kTlBlock) void k_construct_lanes(DevEvent ev, KParams kp, Scratch sc) {
  extern __shared__ __align__(16) int32_t s_hits[];  // LDSH: [A][kHitStride] row slots
  __shared__ float s_x[TPC_MAX_ROWS];
  if (event_bad(sc.counters)) return;
  for (int i = threadIdx.x; i < kp.n_rows; i += kTlBlock) s_x[i] = kp.row_x[i];
  __syncthreads();
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int nr = kp.n_rows;
  Work wk;

  // XCD-aware mapping: workgroups are spread round-robin over the 8 XCDs,
  // each with its own L2.  Blocks b = g (mod G) take the tracklets of the
  // sectors s = g (mod G), G = min(8, sectors), so one XCD reads the grids
  // of only a few sectors.  Only the first A lanes of a wave take tracklets:
  // the constructor's time is the critical path of its longest tracklets, and
  // a wave with fewer lanes waits on fewer scattered loads per step (A is a
  // tuning knob).  Any mapping gives the same results.
  const int G = min(8, ev.n_sectors);
  const int A = min(max(kp.construct_lanes, 1), kTlBlock);
  const int grp = blockIdx.x % G;
  const int blocks_g = ((int)gridDim.x - grp + G - 1) / G;
  const int lanes_g = blocks_g * A;
  int total_g = 0;
  for (int sct = grp; sct < ev.n_sectors; sct += G)
    total_g += sc.row_cnt[(sct + 1) * nr] - sc.row_cnt[sct * nr];
  // k-th tracklet of this group -> tracklet index (sectors are contiguous)
  auto group_tracklet = [&](int k) {
    for (int sct = grp; sct < ev.n_sectors; sct += G) {
      const int o = sc.row_cnt[sct * nr], c = sc.row_cnt[(sct + 1) * nr] - o;
      if (k < c) return min(o + k, n_tl);
      k -= c;
    }
    return n_tl;
  };
  int kg = (int)threadIdx.x < A ? (int)(blockIdx.x / G) * A + (int)threadIdx.x : total_g;
  int t = kg < total_g ? group_tracklet(kg) : n_tl;
  Lane<ENDS, LDSH> ln;
  if constexpr (LDSH) ln.H = s_hits + min((int)threadIdx.x, A - 1) * kHitStride;
  RowGrid gn;  // grid header of the next extension row, loaded one step early
  if (t < n_tl) ln.begin(t, ev, kp, sc, s_x);
  while (t < n_tl) {
    bool finish = ln.dropped;
    if (!finish) {
      const RowGrid g = gn;
      auto search = [&](float& my, float& mz) {
        return search_row(sc, g, g.bin_base - (ln.rsb + ln.r), ln.s, kp, my, mz, wk);
      };
      finish = ln.step(ev, kp, sc, s_x, search, wk);
      if (!finish && ln.extending()) gn = sc.grid[ln.rsb + ln.r];
    }
    if (finish) {
      ln.emit(sc);
      // refill from this group's queue (only when it has more tracklets than lanes)
      kg = lanes_g < total_g ? lanes_g + atomicAdd(&sc.counters[C_QUEUE + grp], 1) : total_g;
      t = kg < total_g ? group_tracklet(kg) : n_tl;
      if (t < n_tl) ln.begin(t, ev, kp, sc, s_x);
    }
  }
  flush_work(wk, sc);
}

// ------------------------------------------------------------------ selection
//
// k_own: per sector, in LDS.  Clusters of different sectors never share a
// tracklet, so the per-cluster argmax of the weights (section 1's selection,
// section 3.1's weight) is a sector-local reduction: a workgroup holds the
// owner keys of a chunk of the sector's clusters in LDS, applies every
// competing tracklet's key with LDS atomics, writes the chunk's keys out and
// counts, per tracklet, the clusters whose key is its own.  A sector larger
// than one chunk is split over several chunks (row ranges); the counts of a
// tracklet are then summed over its chunks.

__device__ __forceinline__ unsigned int order_bits(float w) {
  const unsigned int u = __float_as_uint(w + 0.f);  // -0 -> +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kOwnBlock = 512;
constexpr int kOwnChunk = 4096;   // clusters per chunk at most (KParams::own_chunk)
constexpr int kOwnTable = 1024;   // tracklets per pass over the hit table
constexpr int kOwnSplit = 32;     // workgroups per sector; chunks are dealt out

// Owner key of tracklet t, 0 if it does not compete: the weight
// w = n (alpha - (chi^2/ndf)/beta) in order-preserving bits above the
// complement of the seed id, so that equal weights go to the smaller id.
__device__ __forceinline__ unsigned long long tracklet_key(const KParams& kp, const Scratch& sc,
                                                           int t) {
  const int n = sc.n[t];
  const float qpt = sc.par[(size_t)t * 6 + 5];
  if (n >= kp.min_clusters && (kp.bz == 0.f || fabsf(qpt) <= kp.max_qpt)) {
    const float w = (float)n * (kp.alpha - (sc.chi2[t] / (float)sc.ndf[t]) / kp.beta);
    return ((unsigned long long)order_bits(w) << 32) |
           (unsigned long long)(0xFFFFFFFFu - (unsigned int)sc.seeds[t]);
  }
  return 0ull;
}

__global__ __launch_bounds__(kOwnBlock) void k_own(DevEvent ev, KParams kp, Scratch sc) {
  __shared__ unsigned long long s_own[kOwnChunk];
  __shared__ unsigned long long s_key[kOwnTable];
  __shared__ int s_lh[kOwnTable];   // row_lo | row_hi << 16, clipped to the chunk's rows
  __shared__ int s_cnt[kOwnTable];
  __shared__ int s_rows[2];
  if (event_bad(sc.counters)) return;
  const int nr = kp.n_rows;
  // workgroup -> (sector, first chunk): a grid of (sectors, kOwnSplit), every
  // sector's first workgroups first, or with KParams::own_by_sector a grid of
  // sectors x kOwnSplit in which a sector's workgroups are consecutive
  const int s = kp.own_by_sector ? (int)blockIdx.x / kOwnSplit : (int)blockIdx.x;
  const int split = kp.own_by_sector ? (int)blockIdx.x % kOwnSplit : (int)blockIdx.y;
  const int tid = threadIdx.x;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int t0 = min(sc.row_cnt[s * nr], n_tl), t1 = min(sc.row_cnt[(s + 1) * nr], n_tl);
  const int c0 = ev.ro[s * nr], c1 = ev.ro[(s + 1) * nr];
  const int chunk = min(max(kp.own_chunk, 256), kOwnChunk);
  const int nch = (c1 - c0 + chunk - 1) / chunk;
  for (int ch = split; ch < nch; ch += kOwnSplit) {
    const int cb = c0 + ch * chunk, ce = min(cb + chunk, c1);
    // rows of the sector with clusters in [cb, ce)
    if (tid == 0) {
      s_rows[0] = nr;
      s_rows[1] = -1;
    }
    for (int i = tid; i < ce - cb; i += kOwnBlock) s_own[i] = 0ull;
    __syncthreads();
    for (int r = tid; r < nr; r += kOwnBlock) {
      const int lo = ev.ro[s * nr + r], hi = ev.ro[s * nr + r + 1];
      if (hi > lo && hi > cb && lo < ce) {
        atomicMin(&s_rows[0], r);
        atomicMax(&s_rows[1], r);
      }
    }
    __syncthreads();
    const int rlo = s_rows[0], rhi = s_rows[1];
    // only the 4-row groups of the chunk's rows are read
    const int q0 = rlo >> 2, nq = (rhi >> 2) - q0 + 1;
    for (int pass = 0; pass < 2; ++pass) {  // 0: owner keys, 1: owned counts
      for (int tb = t0; tb < t1; tb += kOwnTable) {
        const int nb = min(kOwnTable, t1 - tb);
        for (int k = tid; k < nb; k += kOwnBlock) {
          const int t = tb + k;
          const unsigned long long key = tracklet_key(kp, sc, t);
          const int lo = max(max(sc.row_lo[t], rlo), 0);
          const int hi = min(min(sc.row_hi[t], rhi), kHitStride - 1);
          s_key[k] = key;
          s_lh[k] = (key != 0ull && lo <= hi) ? (lo | (hi << 16)) : -1;
          s_cnt[k] = 0;
          if (pass == 0 && ch == 0) sc.key[t] = key;
        }
        __syncthreads();
        // (tracklet, 4 rows) elements of the batch; four loads in flight per lane
        const int ne = nb * nq;
        for (int e0 = 0; e0 < ne; e0 += 4 * kOwnBlock) {
          int4 h[4];
          int lh[4], kk[4], rr[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kOwnBlock + tid;
            lh[u] = -1;
            kk[u] = 0;
            rr[u] = 0;
            h[u] = make_int4(-1, -1, -1, -1);
            if (e < ne) {
              const int k = e / nq, r0 = (q0 + (e - k * nq)) * 4;
              const int v = s_lh[k];
              kk[u] = k;
              rr[u] = r0;
              if (v >= 0 && r0 <= (v >> 16) && r0 + 3 >= (v & 0xFFFF)) {
                lh[u] = v;
                h[u] = *reinterpret_cast<const int4*>(sc.hits + (size_t)(tb + k) * kHitStride + r0);
              }
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (lh[u] < 0) continue;
            const int k = kk[u], r0 = rr[u];
            const int lo = lh[u] & 0xFFFF, hi = lh[u] >> 16;
            const unsigned long long key = s_key[k];
            const int hv[4] = {h[u].x, h[u].y, h[u].z, h[u].w};
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int r = r0 + j, c = hv[j];
              if (r < lo || r > hi || c < cb || c >= ce) continue;
              if (pass == 0)
                atomicMax(&s_own[c - cb], key);
              else
                cnt += s_own[c - cb] == key ? 1 : 0;
            }
            if (cnt) atomicAdd(&s_cnt[k], cnt);
          }
        }
        __syncthreads();
        if (pass == 1) {
          for (int k = tid; k < nb; k += kOwnBlock) {
            const int v = s_cnt[k];
            if (nch == 1)
              sc.owned[tb + k] = v;
            else if (v)
              atomicAdd(&sc.owned[tb + k], v);
          }
        }
        __syncthreads();
      }
      if (pass == 0)
        for (int i = tid; i < ce - cb; i += kOwnBlock) sc.own[cb + i] = s_own[i];
      __syncthreads();
    }
  }
}

// Track index and cluster offset of every kept tracklet, in two passes over
// spans of kSpan tracklets: k_tl_reduce sums each span, k_tl_scan adds the
// sums of the spans before it to a scan of its own span.
constexpr int kSpanPer = 4;
constexpr int kSpan = kScanBlock * kSpanPer;

__global__ __launch_bounds__(kScanBlock) void k_tl_reduce(Scratch sc, int min_clusters) {
  __shared__ int s_w[kScanBlock / 64];
  if (event_bad(sc.counters)) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int base = blockIdx.x * kSpan + threadIdx.x * kSpanPer;
  int st = 0, so = 0;
#pragma unroll
  for (int q = 0; q < kSpanPer; ++q) {
    const int i = base + q;
    if (i < n_tl) {
      const int o = sc.owned[i];
      const bool kept = o >= min_clusters;  // section 5: at least 30 owned clusters
      st += kept ? 1 : 0;
      so += kept ? o : 0;
    }
  }
  int tt, to;
  block_excl_scan<kScanBlock>(st, s_w, &tt);
  block_excl_scan<kScanBlock>(so, s_w, &to);
  if (threadIdx.x == 0) {
    sc.span_sum[2 * blockIdx.x] = tt;
    sc.span_sum[2 * blockIdx.x + 1] = to;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_tl_scan(Scratch sc, int min_clusters,
                                                        int cap_tracks, int cap_track_clusters) {
  __shared__ int s_w[kScanBlock / 64];
  if (event_bad(sc.counters)) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int tid = threadIdx.x;
  // offsets of this span: sums of the spans before it
  int pt = 0, po = 0;
  for (int j = tid; j < (int)blockIdx.x; j += kScanBlock) {
    pt += sc.span_sum[2 * j];
    po += sc.span_sum[2 * j + 1];
  }
  int off_t, off_o;
  block_excl_scan<kScanBlock>(pt, s_w, &off_t);
  block_excl_scan<kScanBlock>(po, s_w, &off_o);
  const int base = blockIdx.x * kSpan + tid * kSpanPer;
  int kv[kSpanPer], ov[kSpanPer];
  int st = 0, so = 0;
#pragma unroll
  for (int q = 0; q < kSpanPer; ++q) {
    const int i = base + q;
    const int o = i < n_tl ? sc.owned[i] : 0;
    kv[q] = o >= min_clusters ? 1 : 0;
    ov[q] = kv[q] ? o : 0;
    st += kv[q];
    so += ov[q];
  }
  int tt, to;
  int et = block_excl_scan<kScanBlock>(st, s_w, &tt) + off_t;
  int eo = block_excl_scan<kScanBlock>(so, s_w, &to) + off_o;
#pragma unroll
  for (int q = 0; q < kSpanPer; ++q) {
    const int i = base + q;
    if (i < n_tl) {
      sc.trk_idx[i] = et;
      sc.trk_off[i] = eo;
      sc.kept[i] = kv[q];
      sc.owned[i] = ov[q];
    }
    et += kv[q];
    eo += ov[q];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 0) {
    const int nt = off_t + tt, nc = off_o + to;
    sc.counters[C_TRACKS] = nt;
    sc.counters[C_TRACK_CLUSTERS] = nc;
    if (nt > cap_tracks || nc > cap_track_clusters) atomicOr(&sc.counters[C_ERR], E_CAPACITY);
  }
}

__global__ __launch_bounds__(kGridBlock) void k_output(DevEvent ev, KParams kp, Scratch sc,
                                                       Outputs out) {
  if (__builtin_nontemporal_load(&sc.counters[C_ERR]) != 0) {
    // bad input, capacity exceeded or tracklet overflow: nothing is written
    return;
  }
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  const int n_cl = ev.n_dev ? *ev.n_dev : ev.n_clusters;
  const int lane = threadIdx.x & 63;
  const int wpb = kGridBlock / 64;
  const unsigned long long lt = (1ull << lane) - 1ull;
  constexpr int kChunks = (kHitStride + 63) / 64;  // 64-row pieces of a hit row list
  for (int t = blockIdx.x * wpb + (threadIdx.x >> 6); t < n_tl; t += gridDim.x * wpb) {
    // the tracklet's fields are loaded with its flag (they exist for every
    // tracklet), then every piece's hits at once and their owner keys at
    // once: three waits per kept tracklet instead of two per piece
    const bool kept = sc.kept[t] != 0;
    const int i = sc.trk_idx[t];
    int off = sc.trk_off[t];
    const unsigned long long key = sc.key[t];
    const int lo = max(sc.row_lo[t], 0), hi = min(sc.row_hi[t], kHitStride - 1);
    if (!kept) continue;  // wave-uniform
    const int32_t* H = sc.hits + (size_t)t * kHitStride;
    int c[kChunks];
#pragma unroll
    for (int u = 0; u < kChunks; ++u) {
      const int r = lo + u * 64 + lane;
      c[u] = r <= hi ? H[r] : -1;
    }
    bool mine[kChunks];
#pragma unroll
    for (int u = 0; u < kChunks; ++u) mine[u] = c[u] >= 0 && c[u] < n_cl && sc.own[c[u]] == key;
#pragma unroll
    for (int u = 0; u < kChunks; ++u) {
      const unsigned long long m = __ballot(mine[u]);
      if (mine[u]) {
        const int k = __popcll(m & lt);
        out.track_cluster[off + k] = c[u];
        out.cluster_track[c[u]] = i;
      }
      off += __popcll(m);
    }
    if (lane < 8) {
      const float* P = sc.par + (size_t)t * 6;
      float v;
      if (lane < 6) v = P[lane];
      else if (lane == 6) v = sc.chi2[t];
      else v = (float)sc.ndf[t];
      out.track_par[(size_t)i * 8 + lane] = v;
    } else if (lane < 12) {
      int v;
      const int q = lane - 8;
      if (q == 0) v = ev.sector_id[sc.seed_rs[t] / kp.n_rows];
      else if (q == 1) v = sc.owned[t];
      else if (q == 2) v = sc.trk_off[t];
      else v = sc.seeds[t];
      out.track_meta[(size_t)i * 4 + q] = v;
    }
  }
}

// ------------------------------------------------------------------ global tracking
//
// Section 5: the end of a sector track that leaves its sector through a side
// edge is prolonged into the neighbouring sector.  One lane per slot
// q = 2 * tracklet + end of a kept tracklet (end 0 = inner, 1 = outer):
//   1. from the end state recorded by the constructor, helix steps away from
//      the track through the own sector's rows, without search, until the
//      track is outside the trapezoid; reaching the first/last row, the
//      |sin phi| limit or |z| > z_max ends it without prolongation;
//   2. the neighbour on that side -- same half of the 2 x 18 layout, index
//      +1 (y > 0) or -1 (mod 18) -- if the event holds it (its first slot with
//      that id); the state at the last row inside is rotated into its frame;
//   3. the construction's extension continues there, row by row in the same
//      direction (chi^2 gate, stop after more than max_miss consecutive
//      misses), among the clusters no sector track owns.  A collected
//      cluster is claimed with an atomic minimum of q, so that one collected
//      by several prolongations goes to the smallest (seed id, end): tracklet
//      indices follow the seed ids.
// k_pro_own then counts the clusters each slot owns, the selection's scan
// numbers the slots that own at least one, and k_pro_output writes them in
// (track, end) order.

__global__ __launch_bounds__(kGridBlock) void k_pro_init(DevEvent ev, KParams kp, Scratch sc,
                                                         GlobalScratch gs,
                                                         const int32_t* cluster_track) {
  __shared__ int s_p2s[kLayoutSectors];
  const int n_cl = ev.n_dev ? *ev.n_dev : ev.n_clusters;
  const int stride = gridDim.x * kGridBlock;
  for (int i = blockIdx.x * kGridBlock + threadIdx.x; i < n_cl; i += stride)
    gs.claim[i] = 0x7fffffff;
  // the sector tracker's ownership into the grid records' spare word (for
  // the prolongations' free-cluster test), row slot by row slot: a row's
  // first bins[ny * nz] records are its clusters.  Nothing to do after an
  // error of the tracker (no prolongation then) or without prolongations.
  if (cluster_track && sc.counters[C_ERR] == 0) {
    const int R = ev.n_sectors * kp.n_rows;
    for (int rs = blockIdx.x; rs < R; rs += gridDim.x) {
      const RowGrid g = sc.grid[rs];
      if (g.n == 0) continue;
      const int cnt = sc.bins[g.bin_base + g.ny * g.nz];
      GridRec* rec = sc.g_rec + ev.ro[rs];
      for (int j = threadIdx.x; j < cnt; j += kGridBlock)
        rec[j].pad = cluster_track[rec[j].id] >= 0 ? 1 : 0;
    }
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x < kLayoutSectors) s_p2s[threadIdx.x] = 0x7fffffff;
  __syncthreads();
  for (int sl = threadIdx.x; sl < ev.n_sectors; sl += kGridBlock) {
    const int ph = ev.sector_id[sl];
    if (ph >= 0 && ph < kLayoutSectors) atomicMin(&s_p2s[ph], sl);
  }
  __syncthreads();
  if (threadIdx.x < kLayoutSectors) {
    const int v = s_p2s[threadIdx.x];
    gs.p2s[threadIdx.x] = v == 0x7fffffff ? -1 : v;
  }
  if (threadIdx.x < C_COUNT) {
    // after any error of the sector tracker (its outputs are then not
    // written) there are no slots: every later kernel does nothing
    const int err = sc.counters[C_ERR];
    int v = 0;
    if (threadIdx.x == C_ERR) v = err;
    else if (threadIdx.x == C_SEEDS) v = err ? 0 : 2 * min(sc.counters[C_SEEDS], sc.cap_tl);
    gs.counters[threadIdx.x] = v;
  }
}

// The end states of the tracks at their clusters' rows: each pass stored its
// state when it ended, some rows without a cluster beyond its last cluster,
// and one helix step carries it back.  Also lists the tracks' slots (two
// per kept tracklet) in track order.
__global__ __launch_bounds__(kGridBlock) void k_ends(KParams kp, Scratch sc, GlobalScratch gs) {
  __shared__ float s_x[TPC_MAX_ROWS];
  for (int i = threadIdx.x; i < kp.n_rows; i += kGridBlock) s_x[i] = kp.row_x[i];
  __syncthreads();
  if (event_bad(sc.counters) || __builtin_nontemporal_load(&gs.counters[C_SEEDS]) == 0) return;
  const int n_tl = min(sc.counters[C_SEEDS], sc.cap_tl);
  for (int q = blockIdx.x * kGridBlock + threadIdx.x; q < 2 * n_tl; q += gridDim.x * kGridBlock) {
    const int t = q >> 1, e = q & 1;
    if (!sc.kept[t]) continue;
    gs.act[2 * sc.trk_idx[t] + e] = q;
    float* E = sc.ends + (size_t)q * kEndStride;
    KState s;
    load_end(E, s);
    const bool ok = propagate(s, s_x[e ? sc.row_hi[t] : sc.row_lo[t]], kp);
    if (ok) store_end(E, s);
    E[kEndValid] = ok ? 1.f : 0.f;
  }
}

// A cluster no sector track owns: k_pro_init copies the sector tracker's
// cluster_track into the grid records' spare word (1 = owned), so the test
// reads the record the search already holds.
struct FreeCluster {
  __device__ bool operator()(const GridRec& v) const { return v.pad == 0; }
};

// Prolongation of slot q; returns the number of clusters collected.
__device__ int prolong_slot(int q, const DevEvent& ev, const KParams& kp, const Scratch& sc,
                            const GlobalScratch& gs, const float* s_x) {
  const int t = q >> 1, e = q & 1, dir = e ? 1 : -1, nr = kp.n_rows;
  const int row = e ? sc.row_hi[t] : sc.row_lo[t];
  const float* E = sc.ends + (size_t)q * kEndStride;
  if (E[kEndValid] == 0.f) return 0;
  KState s;
  load_end(E, s);
  // 1. own sector, no search, until the track is outside the trapezoid: the
  //    checks need only the parameters, the covariance is carried once, to
  //    the last row inside
  HelixPar h{s.x, s.y, s.z, s.sp, s.tl, s.qpt};
  int r = row + dir, last_r = row;
  bool left = false, up = false;
  for (; r >= 0 && r < nr; r += dir) {
    if (!step_par(h, s_x[r], kp)) return 0;
    if (fabsf(h.z) > kp.z_max) return 0;
    if (fabsf(h.y) > s_x[r] * kp.tan_half) {
      left = true;
      up = h.y > 0.f;
      break;
    }
    last_r = r;
  }
  if (!left) return 0;
  if (last_r != row && !propagate(s, s_x[last_r], kp)) return 0;
  // 2. the neighbour on that side
  const int phys = ev.sector_id[sc.seed_rs[t] / nr];
  if (phys < 0 || phys >= kLayoutSectors) return 0;
  const int nphys = (phys / 18) * 18 + (phys % 18 + (up ? 1 : 17)) % 18;
  const int ns = gs.p2s[nphys];
  if (ns < 0) return 0;
  if (!rotate(s, kp.rot_c, up ? kp.rot_s : -kp.rot_s, kp)) return 0;
  if (fabsf(s.sp) > kp.max_sinphi) return 0;
  // 3. extension in the neighbour from the first row beyond x
  r = dir < 0 ? nr - 1 : 0;
  if (dir < 0)
    while (r >= 0 && s_x[r] >= s.x) --r;
  else
    while (r < nr && s_x[r] <= s.x) ++r;
  int32_t* H = gs.hit + (size_t)q * kHitStride;
  float* P = gs.par + (size_t)q * 8;
  const FreeCluster free_only{};
  Work wk;
  int misses = 0, n = 0;
  float chi2 = 0.f;
  RowGrid gn;  // grid header of row r, loaded one step ahead
  if (r >= 0 && r < nr) gn = sc.grid[ns * nr + r];
  for (; r >= 0 && r < nr; r += dir) {
    const RowGrid g = gn;
    if (r + dir >= 0 && r + dir < nr) gn = sc.grid[ns * nr + r + dir];
    if (!propagate(s, s_x[r], kp)) break;
    if (fabsf(s.z) > kp.z_max) break;
    int h = -1;
    float my = 0.f, mz = 0.f;
    if (!(fabsf(s.y) > s_x[r] * kp.tan_half))
      h = search_row(sc, g, g.bin_base - (ns * nr + r), s, kp, my, mz, wk, free_only);
    if (h >= 0) {
      chi2 += kf_update(s, my, mz, kp);
      H[n++] = h;
      atomicMin(&gs.claim[h], q);
      P[0] = s.x; P[1] = s.y; P[2] = s.z; P[3] = s.sp; P[4] = s.tl; P[5] = s.qpt;
      misses = 0;
    } else if (++misses > kp.max_miss) {
      break;
    }
  }
  if (n > 0) {
    P[6] = chi2;
    P[7] = (float)(2 * n);
    gs.nslot[q] = ns;
  }
  return n;
}

__global__ __launch_bounds__(kGridBlock) void k_prolong(DevEvent ev, KParams kp, Scratch sc,
                                                        GlobalScratch gs) {
  __shared__ float s_x[TPC_MAX_ROWS];
  for (int i = threadIdx.x; i < kp.n_rows; i += kGridBlock) s_x[i] = kp.row_x[i];
  __syncthreads();
  if (event_bad(gs.counters) || gs.counters[C_SEEDS] == 0) return;
  // the kept tracklets' slots only (other slots are never read as collected)
  const int n_act = 2 * sc.counters[C_TRACKS];
  for (int i = blockIdx.x * kGridBlock + threadIdx.x; i < n_act; i += gridDim.x * kGridBlock) {
    const int q = gs.act[i];
    gs.n[q] = prolong_slot(q, ev, kp, sc, gs, s_x);
  }
}

__global__ __launch_bounds__(kGridBlock) void k_pro_own(Scratch sc, GlobalScratch gs) {
  if (event_bad(gs.counters)) return;
  const int n_slots = gs.counters[C_SEEDS];
  for (int q = blockIdx.x * kGridBlock + threadIdx.x; q < n_slots; q += gridDim.x * kGridBlock) {
    const int n = sc.kept[q >> 1] ? gs.n[q] : 0;
    const int32_t* H = gs.hit + (size_t)q * kHitStride;
    int o = 0;
    for (int j = 0; j < n; ++j) o += gs.claim[H[j]] == q ? 1 : 0;
    gs.owned[q] = o;
  }
}

// One wave per slot: the owned clusters in the order met, state, meta.
__global__ __launch_bounds__(kGridBlock) void k_pro_output(DevEvent ev, Scratch sc,
                                                           GlobalScratch gs, ProOutputs po) {
  if (__builtin_nontemporal_load(&gs.counters[C_ERR]) != 0) return;
  const int n_slots = gs.counters[C_SEEDS];
  const int lane = threadIdx.x & 63;
  const int wpb = kGridBlock / 64;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int q = blockIdx.x * wpb + (threadIdx.x >> 6); q < n_slots; q += gridDim.x * wpb) {
    if (!gs.kept[q]) continue;  // wave-uniform
    const int i = gs.idx[q];
    int off = gs.off[q];
    const int n = min(gs.n[q], kHitStride);
    const int32_t* H = gs.hit + (size_t)q * kHitStride;
    for (int j0 = 0; j0 < n; j0 += 64) {  // wave-uniform trip count
      const int j = j0 + lane;
      const int c = j < n ? H[j] : -1;
      const bool mine = c >= 0 && gs.claim[c] == q;
      const unsigned long long m = __ballot(mine);
      if (mine) po.cluster[off + __popcll(m & lt)] = c;
      off += __popcll(m);
    }
    if (lane < 8) {
      po.par[(size_t)i * 8 + lane] = gs.par[(size_t)q * 8 + lane];
    } else if (lane < 13) {
      const int k = lane - 8;
      int v;
      if (k == 0) v = sc.trk_idx[q >> 1];
      else if (k == 1) v = q & 1;
      else if (k == 2) v = ev.sector_id[gs.nslot[q]];
      else if (k == 3) v = gs.owned[q];
      else v = gs.off[q];
      po.meta[(size_t)i * 5 + k] = v;
    }
  }
}

// ------------------------------------------------------------------ track merger
//
// Section 1's chain: the sector tracks of one particle are joined and every
// joined track is refitted from its cluster list alone, so that the same
// clusters give the same fit whatever the sector tracker computed on the way
// (section 3.3).  A join links the outer end of track A (the outward filter
// at its outermost cluster) to the inner end of track B (the inward fit at
// its innermost cluster) in a side neighbour of A's sector or in its
// membrane partner, if B starts farther from the beam than A ends: A's end
// is rotated into B's frame and propagated to B's x, and the two
// independent estimates give chi^2 = d^T (C_A + C_B)^-1 d over the five
// parameters; A and B are linked if each is the other's best candidate
// under the cut (smallest chi^2, then smallest track).  One lane per track
// A finds its best B and offers itself to every candidate B with a 64-bit
// atomic minimum of (chi^2 bits, A).

// Whole sector widths from the frame of sector id p to that of q (both in
// the 2 x 18 layout), in [-9, 8].
__device__ __forceinline__ int frame_steps(int p, int q) {
  int k = (q % 18) - (p % 18);
  if (k > 8) k -= 18;
  if (k < -9) k += 18;
  return k;
}

__device__ __forceinline__ bool rotate_steps(KState& s, int k, const KParams& kp) {
  return k == 0 || rotate(s, kp.rot_tab[k + 9][0], kp.rot_tab[k + 9][1], kp);
}

// Track i's tracklet (its two slots were listed in track order by k_ends).
__device__ __forceinline__ int tl_of_track(const GlobalScratch& gs, int i) {
  return gs.act[2 * i] >> 1;
}

__global__ __launch_bounds__(kGridBlock) void k_mrg_init(DevEvent ev, KParams kp, Scratch sc,
                                                         GlobalScratch gs, MergeScratch ms) {
  if (event_bad(sc.counters)) return;
  const int err = sc.counters[C_ERR];
  const int nt = err ? 0 : sc.counters[C_TRACKS];
  const int nr = kp.n_rows;
  const int tid = blockIdx.x * kGridBlock + threadIdx.x, stride = gridDim.x * kGridBlock;
  if (tid < C_COUNT) {
    int v = 0;
    if (tid == C_ERR) v = err;
    else if (tid == C_SEEDS) v = nt;
    ms.counters[tid] = v;
  }
  // first track of each slot: tracks follow the tracklets, in slot order
  for (int sl = tid; sl <= ev.n_sectors; sl += stride) {
    int lo = 0, hi = nt;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sc.seed_rs[tl_of_track(gs, mid)] / nr < sl) lo = mid + 1;
      else hi = mid;
    }
    ms.first[sl] = lo;
  }
  for (int i = tid; i < nt; i += stride) {
    const float* E = sc.ends + (size_t)(2 * tl_of_track(gs, i)) * kEndStride;
    const float4 a = reinterpret_cast<const float4*>(E)[0];
    const float4 b = reinterpret_cast<const float4*>(E)[1];
    ms.sum[2 * i] = make_float4(a.x, a.y, b.x, b.y);
    // var tan(lambda) = C33, var q/pT = C44 (packed elements 9 and 14)
    const double* EC = end_cov(E);
    ms.sum[2 * i + 1] = make_float4((float)EC[9], (float)EC[14], sqrtf(a.x * a.x + a.y * a.y),
                                    E[kEndValid]);
    ms.prev_key[i] = ~0ull;
    ms.prev[i] = -1;
  }
}

// chi^2 of d^T S^-1 d for a symmetric positive-definite S (Cholesky), or -1.
__device__ __forceinline__ float chi2_5(const float d[5], float S[5][5]) {
  float L[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float v = S[i][j];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      if (i == j) {
        if (!(v > 0.f)) return -1.f;
        L[i][i] = sqrtf(v);
      } else {
        L[i][j] = v / L[j][j];
      }
    }
  float chi2 = 0.f, y[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float v = d[i];
#pragma unroll
    for (int q = 0; q < i; ++q) v -= L[i][q] * y[q];
    y[i] = v / L[i][i];
    chi2 += y[i] * y[i];
  }
  return chi2;
}

__device__ __forceinline__ void cov_full(const Cov& C, float M[5][5]) {
  // the join test is a decision: FP32 is enough
  M[0][0] = C.c00; M[1][0] = C.c10; M[1][1] = C.c11; M[2][0] = C.c20; M[2][1] = C.c21;
  M[2][2] = C.c22; M[3][0] = C.c30; M[3][1] = C.c31; M[3][2] = C.c32; M[3][3] = C.c33;
  M[4][0] = C.c40; M[4][1] = C.c41; M[4][2] = C.c42; M[4][3] = C.c43; M[4][4] = C.c44;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i + 1; j < 5; ++j) M[i][j] = M[j][i];
}

// One wave per track A: the lanes take A's candidates in turn; the wave's
// best is the minimum of (chi^2 bits, candidate) over its lanes.
__global__ __launch_bounds__(kGridBlock) void k_mrg_match(DevEvent ev, KParams kp, Scratch sc,
                                                          GlobalScratch gs, MergeScratch ms) {
  if (event_bad(sc.counters)) return;
  const int nt = ms.counters[C_SEEDS];
  const int nr = kp.n_rows;
  const float cut = kp.merge_chi2;
  const int lane = threadIdx.x & 63;
  const int wpb = kGridBlock / 64;
  for (int a = blockIdx.x * wpb + (threadIdx.x >> 6); a < nt; a += gridDim.x * wpb) {
    unsigned long long best = ~0ull;  // (chi^2 bits << 32) | candidate
    const int ta = tl_of_track(gs, a);
    const int sa = sc.seed_rs[ta] / nr;
    const int pa = ev.sector_id[sa];
    const float* EA = sc.ends + (size_t)(2 * ta + 1) * kEndStride;
    if (pa >= 0 && pa < kLayoutSectors && EA[kEndValid] != 0.f) {  // wave-uniform
      KState A;
      load_end(EA, A);
      const float ra = sqrtf(A.x * A.x + A.y * A.y);
      const int half = pa / 18, idx = pa % 18;
      const int cand[3] = {gs.p2s[half * 18 + (idx + 1) % 18], gs.p2s[half * 18 + (idx + 17) % 18],
                           gs.p2s[(pa + 18) % kLayoutSectors]};
      for (int c = 0; c < 3; ++c) {
        const int sb = cand[c];
        if (sb < 0 || sb == sa || (c > 0 && cand[0] == sb) || (c > 1 && cand[1] == sb)) continue;
        KState R = A;  // A's end in B's frame, once per slot
        if (!rotate_steps(R, frame_steps(pa, ev.sector_id[sb]), kp)) continue;
        for (int b = ms.first[sb] + lane; b < ms.first[sb + 1]; b += 64) {
          const float4 u = ms.sum[2 * b], v = ms.sum[2 * b + 1];
          // tan(lambda), q/pT and their variances do not change under rotation
          // and propagation, and d_i^2 / S_ii <= chi^2: exact rejections
          const float dt = u.z - A.tl, dq = u.w - A.qpt;
          if (dt * dt > cut * ((float)A.C.c33 + v.x) || dq * dq > cut * ((float)A.C.c44 + v.y))
            continue;
          if (!(v.z > ra) || v.w == 0.f) continue;  // outward only; valid end
          KState B;
          load_end(sc.ends + (size_t)(2 * tl_of_track(gs, b)) * kEndStride, B);
          KState T = R;
          if (!propagate(T, B.x, kp)) continue;
          float S[5][5], SB[5][5];
          cov_full(T.C, S);
          cov_full(B.C, SB);
#pragma unroll
          for (int i = 0; i < 5; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) S[i][j] += SB[i][j];
          const float d[5] = {B.y - T.y, B.z - T.z, B.sp - T.sp, B.tl - T.tl, B.qpt - T.qpt};
          const float x2 = chi2_5(d, S);
          if (!(x2 >= 0.f) || x2 > cut) continue;
          const unsigned long long hi = (unsigned long long)__float_as_uint(x2) << 32;
          best = min(best, hi | (unsigned int)b);
          atomicMin(&ms.prev_key[b], hi | (unsigned int)a);
        }
      }
    }
    for (int d = 32; d >= 1; d >>= 1) {
      const unsigned long long o = __shfl_xor(best, d, 64);
      best = min(best, o);
    }
    if (lane == 0) ms.best[a] = best == ~0ull ? -1 : (int)(best & 0xffffffffull);
  }
}

__global__ __launch_bounds__(kGridBlock) void k_mrg_link(Scratch sc, MergeScratch ms) {
  if (event_bad(sc.counters)) return;
  const int nt = ms.counters[C_SEEDS];
  for (int a = blockIdx.x * kGridBlock + threadIdx.x; a < nt; a += gridDim.x * kGridBlock) {
    const int b = ms.best[a];
    const bool link = b >= 0 && (int)(ms.prev_key[b] & 0xffffffffull) == a;
    ms.next[a] = link ? b : -1;
    if (link) ms.prev[b] = a;  // b's best predecessor is unique
  }
}

// Chain heads (no predecessor; in a closed chain, its smallest track) and
// the clusters of each chain: the inner prolongation of its first track,
// the tracks' own clusters, the outer prolongation of its last track.
__global__ __launch_bounds__(kGridBlock) void k_mrg_chain(Scratch sc, GlobalScratch gs,
                                                          MergeScratch ms, Outputs out,
                                                          int use_pro) {
  if (event_bad(sc.counters)) return;
  const int nt = ms.counters[C_SEEDS];
  // prolongations whose outputs did not fit were not written: not used
  if (use_pro && gs.counters[C_ERR] != 0) use_pro = 0;
  for (int i = blockIdx.x * kGridBlock + threadIdx.x; i < nt; i += gridDim.x * kGridBlock) {
    bool head = ms.prev[i] < 0;
    if (!head) {
      int j = ms.prev[i], mn = i;
      for (int k = 0; k < nt && j >= 0 && j != i; ++k) {
        mn = min(mn, j);
        j = ms.prev[j];
      }
      head = j == i && mn == i;
    }
    int cnt = 0, nseg = 0;
    if (head) {
      int j = i, last = i;
      do {
        cnt += out.track_meta[(size_t)j * 4 + 1];
        ++nseg;
        last = j;
        j = ms.next[j];
      } while (j >= 0 && j != i && nseg < nt);
      if (use_pro) {
        const int qi = 2 * tl_of_track(gs, i), qo = 2 * tl_of_track(gs, last) + 1;
        if (gs.kept[qi]) cnt += gs.owned[qi];
        if (gs.kept[qo]) cnt += gs.owned[qo];
      }
    }
    ms.cnt[i] = cnt;
    ms.nseg[i] = nseg;
  }
}

// One wave per chain: its list in path order, meta, and the joined index of
// its tracks.
__global__ __launch_bounds__(kGridBlock) void k_mrg_write(DevEvent ev, KParams kp, Scratch sc,
                                                          GlobalScratch gs, MergeScratch ms,
                                                          Outputs out, ProOutputs po, int use_pro,
                                                          MergeOutputs mo) {
  if (__builtin_nontemporal_load(&ms.counters[C_ERR]) != 0) return;
  const int nt = ms.counters[C_SEEDS];
  const int lane = threadIdx.x & 63;
  const int wpb = kGridBlock / 64;
  if (use_pro && gs.counters[C_ERR] != 0) use_pro = 0;  // as in k_mrg_chain
  if (blockIdx.x == 0 && threadIdx.x == 0) ms.loff[ms.counters[C_TRACKS]] =
      ms.counters[C_TRACK_CLUSTERS];
  for (int i = blockIdx.x * wpb + (threadIdx.x >> 6); i < nt; i += gridDim.x * wpb) {
    if (!ms.kept[i]) continue;  // wave-uniform
    const int k = ms.idx[i];
    int off = ms.off[i];
    const int first = off;
    int last = i;
    {  // the last track of the chain
      int j = ms.next[i], n = 1;
      while (j >= 0 && j != i && n < nt) {
        last = j;
        j = ms.next[j];
        ++n;
      }
    }
    if (use_pro) {
      const int q = 2 * tl_of_track(gs, i);
      if (gs.kept[q]) {  // inner prolongation, reversed into path order
        const int pi = gs.idx[q];
        const int n = po.meta[(size_t)pi * 5 + 3], f = po.meta[(size_t)pi * 5 + 4];
        for (int j = lane; j < n; j += 64) mo.cluster[off + j] = po.cluster[f + n - 1 - j];
        off += n;
      }
    }
    int j = i, nseg = 0;
    do {
      const int n = out.track_meta[(size_t)j * 4 + 1], f = out.track_meta[(size_t)j * 4 + 2];
      for (int q = lane; q < n; q += 64) mo.cluster[off + q] = out.track_cluster[f + q];
      if (lane == 0) mo.track_merged[j] = k;
      off += n;
      ++nseg;
      j = ms.next[j];
    } while (j >= 0 && j != i && nseg < nt);
    if (use_pro) {
      const int q = 2 * tl_of_track(gs, last) + 1;
      if (gs.kept[q]) {
        const int pi = gs.idx[q];
        const int n = po.meta[(size_t)pi * 5 + 3], f = po.meta[(size_t)pi * 5 + 4];
        for (int j2 = lane; j2 < n; j2 += 64) mo.cluster[off + j2] = po.cluster[f + j2];
        off += n;
      }
    }
    if (lane < 5) {
      int v;
      if (lane == 0) v = ev.sector_id[sc.seed_rs[tl_of_track(gs, i)] / kp.n_rows];
      else if (lane == 1) v = nseg;
      else if (lane == 2) v = off - first;
      else if (lane == 3) v = first;
      else v = i;
      mo.meta[(size_t)k * 5 + lane] = v;
    }
    if (lane == 0) ms.loff[k] = first;
  }
}

// Row slot of every cluster (one workgroup per row slot); -1 where no row
// holds a cluster index (the offsets were validated by k_grid).
__global__ __launch_bounds__(kGridBlock) void k_rowmap(DevEvent ev, KParams kp, Scratch sc,
                                                      MergeScratch ms) {
  if (event_bad(sc.counters)) return;
  const int rs = blockIdx.x;
  const int a = ev.ro[rs], b = ev.ro[rs + 1];
  for (int c = a + threadIdx.x; c < b; c += kGridBlock) ms.rowslot[c] = rs;
}

// A list entry as the refit reads it: coordinates, row slot and sector slot
// of the cluster (both -1: not a cluster of the event).
__device__ __forceinline__ float4 list_rec(const DevEvent& ev, const MergeScratch& ms, int nr,
                                           int c) {
  const int rs = (c >= 0 && c < ev.n_clusters) ? ms.rowslot[c] : -1;
  return rs >= 0 ? make_float4(ev.y[c], ev.z[c], __int_as_float(rs), __int_as_float(rs / nr))
                 : make_float4(0.f, 0.f, __int_as_float(-1), __int_as_float(-1));
}

// The entries of the lists, gathered once (all entries in parallel), so that
// the refit walks a contiguous 16-byte record per cluster.
__global__ __launch_bounds__(kGridBlock) void k_refit_gather(DevEvent ev, int nr, Scratch sc,
                                                             MergeScratch ms, const int32_t* n_dev,
                                                             int n_host, const int32_t* clusters) {
  if (event_bad(sc.counters)) return;
  if (n_dev && __builtin_nontemporal_load(&ms.counters[C_ERR]) != 0) return;
  const int n = min(n_dev ? *n_dev : n_host, ms.cap_rec);
  for (int e = blockIdx.x * kGridBlock + threadIdx.x; e < n; e += gridDim.x * kGridBlock)
    ms.rec[e] = list_rec(ev, ms, nr, clusters[e]);
}

// The refit of one list (path order, records R[0 .. n)): the seed circle of
// the first run of three or more consecutive clusters of one sector with
// increasing rows (its first min(m, seed_window)), an outward filter to the
// end of the list, an inward fit from the last cluster with a fresh
// covariance over the whole list; frames change by rotations of whole sector
// widths; a cluster whose step fails is skipped.  A list with an entry that
// is not a cluster of the event, or over several sectors one of which has an
// id outside the 2 x 18 layout, fails; the passes check their entries as they
// go (together they see every entry).  P = x, state at the innermost fitted
// cluster, chi^2, ndf (all 0 and frame -1 if the refit fails).  The next
// record is loaded a step ahead.
constexpr int kRefitSlots = 1024;  // sector ids staged in LDS by k_refit

// sid: the sector id of each slot (slot < n_sid; others are read from the
// event).
__device__ void refit_list(const float4* R, int n, const DevEvent& ev, const KParams& kp,
                           const float* s_x, const int32_t* sid, int n_sid, float* P,
                           int32_t* frame) {
  const int nr = kp.n_rows;
  for (int i = 0; i < 8; ++i) P[i] = 0.f;
  *frame = -1;
  if (n < 3) return;
  auto sector_id = [&](int sl) { return sl < n_sid ? sid[sl] : ev.sector_id[sl]; };
  auto slot = [](const float4& r) { return __float_as_int(r.w); };
  bool bad = false, multi = false, bad_id = false;
  int s_first = -1;
  auto note = [&](const float4& r) {  // validity and the sectors seen
    const int sl = slot(r);
    if (sl < 0) {
      bad = true;
      return;
    }
    if (s_first < 0) s_first = sl;
    multi |= sl != s_first;
    const int ph = sector_id(sl);
    bad_id |= ph < 0 || ph >= kLayoutSectors;
  };
  // the seed run: sliding window of three records
  int i0 = -1;
  float4 ra = R[0], rb = R[1];
  note(ra);
  note(rb);
  for (int i = 0; i + 2 < n; ++i) {
    const float4 rc = R[i + 2];
    note(rc);
    const int xa = __float_as_int(ra.z), xb = __float_as_int(rb.z), xc = __float_as_int(rc.z);
    if (xa >= 0 && xb >= 0 && xc >= 0 && slot(rb) == slot(ra) && slot(rc) == slot(ra) &&
        xa < xb && xb < xc) {
      i0 = i;
      break;
    }
    ra = rb;
    rb = rc;
  }
  if (i0 < 0 || bad) return;
  const int rs0 = __float_as_int(R[i0].z), sl0 = slot(R[i0]);
  int m = 1, prs = rs0;
  while (i0 + m < n && m < kp.seed_window) {
    const float4 rm = R[i0 + m];
    const int rs = __float_as_int(rm.z);
    if (rs < 0 || slot(rm) != sl0 || !(rs > prs)) break;
    prs = rs;
    ++m;
  }
  const int ia = i0, ib = i0 + m / 2, ie = i0 + m - 1;
  const float4 A = R[ia], B = R[ib], E = R[ie];
  KState s;
  seed3(s, s_x[__float_as_int(A.z) - sl0 * nr], A.x, A.y, s_x[__float_as_int(B.z) - sl0 * nr], B.x,
        s_x[__float_as_int(E.z) - sl0 * nr], E.x, E.y, kp);
  if (fabsf(s.sp) > kp.max_sinphi) return;
  // outward filter (checks the entries after the seed window's start)
  int fr = sl0, last = i0;
  float4 nx = i0 + 1 < n ? R[i0 + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int j = i0 + 1; j < n; ++j) {
    const float4 cur = nx;
    if (j + 1 < n) nx = R[j + 1];
    const int rs = __float_as_int(cur.z);
    note(cur);
    if (rs < 0 || (multi && bad_id)) continue;
    const int sl = slot(cur);
    KState t = s;
    if (sl != fr && !rotate_steps(t, frame_steps(sector_id(fr), sector_id(sl)), kp)) continue;
    if (!propagate(t, s_x[rs - sl * nr], kp)) continue;
    kf_update(t, cur.x, cur.y, kp);
    s = t;
    fr = sl;
    last = j;
  }
  if (bad || (multi && bad_id)) return;
  // inward fit from the last cluster, fresh covariance
  const float4 L = R[last];
  const int rsl = __float_as_int(L.z);
  KState w;
  w.x = s_x[rsl - slot(L) * nr];
  w.y = L.x;
  w.z = L.y;
  w.sp = s.sp;
  w.tl = s.tl;
  w.qpt = s.qpt;
  reset_cov(w.C, kp);
  float chi2 = 0.f;
  int nn = 1, ifr = slot(L);
  float o[6] = {w.x, w.y, w.z, w.sp, w.tl, w.qpt};
  nx = last > 0 ? R[last - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int j = last - 1; j >= 0; --j) {
    const float4 cur = nx;
    if (j > 0) nx = R[j - 1];
    const int rs = __float_as_int(cur.z);
    const int sl = slot(cur);
    KState t = w;
    if (sl != fr && !rotate_steps(t, frame_steps(sector_id(fr), sector_id(sl)), kp)) continue;
    if (!propagate(t, s_x[rs - sl * nr], kp)) continue;
    chi2 += kf_update(t, cur.x, cur.y, kp);
    w = t;
    fr = sl;
    ++nn;
    ifr = sl;
    o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.sp; o[4] = w.tl; o[5] = w.qpt;
  }
  if (nn < 3) return;
  for (int i = 0; i < 6; ++i) P[i] = o[i];
  P[6] = chi2;
  P[7] = (float)(2 * nn - 5);
  *frame = sector_id(ifr);
}

// One lane per list over the gathered records.  n_lists is read from n_dev
// if given (the merger's own lists), else n_host with list entries clamped
// to [0, min(n_entries, gathered records)).
__global__ __launch_bounds__(kGridBlock) void k_refit(DevEvent ev, KParams kp, Scratch sc,
                                                      MergeScratch ms, const int32_t* n_dev,
                                                      int n_host, int n_entries,
                                                      const int32_t* offsets, float* par,
                                                      int32_t* frame, int32_t* meta_frame) {
  __shared__ float s_x[TPC_MAX_ROWS];
  __shared__ int32_t s_sid[kRefitSlots];  // sector ids of the first slots
  for (int i = threadIdx.x; i < kp.n_rows; i += kGridBlock) s_x[i] = kp.row_x[i];
  const int n_sid = min(ev.n_sectors, kRefitSlots);
  for (int i = threadIdx.x; i < n_sid; i += kGridBlock) s_sid[i] = ev.sector_id[i];
  __syncthreads();
  if (event_bad(sc.counters)) return;
  if (n_dev && __builtin_nontemporal_load(&ms.counters[C_ERR]) != 0) return;
  const int n = n_dev ? *n_dev : n_host;
  const int lim = min(n_entries, ms.cap_rec);
  for (int k = blockIdx.x * kGridBlock + threadIdx.x; k < n; k += gridDim.x * kGridBlock) {
    int a = offsets[k], b = offsets[k + 1];
    a = clampi(a, 0, lim);
    b = clampi(b, a, lim);
    float P[8];
    int32_t f;
    refit_list(ms.rec + a, b - a, ev, kp, s_x, s_sid, n_sid, P, &f);
    for (int i = 0; i < 8; ++i) par[(size_t)k * 8 + i] = P[i];
    if (frame) frame[k] = f;
    if (meta_frame && f >= 0) meta_frame[(size_t)k * 5] = f;
  }
}

// ------------------------------------------------------------------ batches
//
// A batch is tracked as one event whose sector slots are those of all its
// events side by side: sectors never interact, and every tie is broken by
// comparing cluster indices that keep their order within an event, so each
// event's tracks are exactly those it gets alone.

__global__ __launch_bounds__(kGridBlock) void k_batch_gather(BatchBuffers bb, int32_t* counters,
                                                             int n_rows, int n_total,
                                                             int s_total) {
  const BatchEventDesc d = bb.desc[blockIdx.y];
  const int stride = gridDim.x * kGridBlock;
  {  // each event's own offsets must be a partition of [0, n_clusters]
    const int nro_ = d.n_sectors * n_rows;
    for (int r = blockIdx.x * kGridBlock + threadIdx.x; r <= nro_; r += stride) {
      const int v = d.ro[r];
      bool bad = v < 0 || v > d.n_clusters || (r < nro_ && d.ro[r + 1] < v) ||
                 (r == 0 && v != 0) || (r == nro_ && v != d.n_clusters);
      if (bad) atomicOr(&counters[C_ERR], E_OFFSETS);
    }
  }
  for (int i = blockIdx.x * kGridBlock + threadIdx.x; i < d.n_clusters; i += stride) {
    bb.y[d.cbase + i] = d.y[i];
    bb.z[d.cbase + i] = d.z[i];
  }
  const int nro = d.n_sectors * n_rows;
  for (int r = blockIdx.x * kGridBlock + threadIdx.x; r < nro; r += stride)
    bb.ro[d.sbase * n_rows + r] = d.ro[r] + d.cbase;
  for (int q = blockIdx.x * kGridBlock + threadIdx.x; q < d.n_sectors; q += stride)
    bb.sector_id[d.sbase + q] = d.sector_id[q];
  if (blockIdx.y == gridDim.y - 1 && blockIdx.x == 0 && threadIdx.x == 0)
    bb.ro[s_total * n_rows] = d.ro[nro] + d.cbase;  // == n_total when offsets are valid
}

// First track whose seed (an event-global index of the batch) is >= c.
__device__ __forceinline__ int first_track_from(const int32_t* meta, int n_tracks, int c) {
  int lo = 0, hi = n_tracks;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (meta[(size_t)mid * 4 + 3] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kGridBlock) void k_batch_scatter(BatchBuffers bb, Scratch sc) {
  if (__builtin_nontemporal_load(&sc.counters[C_ERR]) != 0) return;
  const int e = blockIdx.y;
  const BatchEventDesc d = bb.desc[e];
  const int nt_all = sc.counters[C_TRACKS];
  const int nc_all = sc.counters[C_TRACK_CLUSTERS];
  const int t0 = first_track_from(bb.meta, nt_all, d.cbase);
  const int t1 = first_track_from(bb.meta, nt_all, d.cbase + d.n_clusters);
  const int o0 = t0 < nt_all ? bb.meta[(size_t)t0 * 4 + 2] : nc_all;
  const int o1 = t1 < nt_all ? bb.meta[(size_t)t1 * 4 + 2] : nc_all;
  const int nt = t1 - t0, nc = o1 - o0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bb.ev_counts[2 * e] = nt;
    bb.ev_counts[2 * e + 1] = nc;
  }
  if (nt > d.cap_tracks || nc > d.cap_track_clusters) return;  // reported, nothing written
  const int stride = gridDim.x * kGridBlock;
  const int tid = blockIdx.x * kGridBlock + threadIdx.x;
  for (int j = tid; j < nt * 8; j += stride) d.track_par[j] = bb.par[(size_t)t0 * 8 + j];
  for (int j = tid; j < nt; j += stride) {
    const int32_t* m = bb.meta + (size_t)(t0 + j) * 4;
    int32_t* o = d.track_meta + (size_t)j * 4;
    o[0] = m[0];
    o[1] = m[1];
    o[2] = m[2] - o0;
    o[3] = m[3] - d.cbase;
  }
  for (int j = tid; j < nc; j += stride) d.track_cluster[j] = bb.tcl[o0 + j] - d.cbase;
  for (int i = tid; i < d.n_clusters; i += stride) {
    const int v = bb.ctr[d.cbase + i];
    d.cluster_track[i] = v < 0 ? -1 : v - t0;
  }
}

hipError_t enqueue_batch_gather(const BatchBuffers& bb, const Scratch& sc, int n_events,
                                int n_rows, int n_total, int s_total, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, sc.counters);
  hipLaunchKernelGGL(k_batch_gather, dim3(64, n_events), dim3(kGridBlock), 0, st, bb,
                     sc.counters, n_rows, n_total, s_total);
  return hipGetLastError();
}

hipError_t enqueue_batch_scatter(const BatchBuffers& bb, const Scratch& sc, int n_events,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_batch_scatter, dim3(64, n_events), dim3(kGridBlock), 0, st, bb, sc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host side

static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ static scratch
//
// The scratch of tpc_track_event_noalloc, for callers that cannot allocate:
// one array per GPU, held until the process ends.  In host code the name
// `scratch` is a host-side stand-in, not a device address: the address on
// each device comes from hipGetSymbolAddress, resolved once per device (with
// that device current) by static_scratch_init, and only that pointer is
// handed to the kernels.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

size_t scratch_bytes(int64_t N, int64_t R, int64_t T) {
  size_t b = 0;
  b += align_up(sizeof(int32_t) * C_COUNT);
  b += align_up(sizeof(RowGrid) * R);
  b += align_up(sizeof(int32_t) * (N + R + 1));
  b += align_up(sizeof(GridRec) * N);
  b += align_up(sizeof(int32_t) * N) * 5;  // up, dn, up2, dn2 + start (bytes, padded)
  b += align_up(sizeof(unsigned long long) * N);
  b += align_up(sizeof(int32_t) * (R + 1));
  b += align_up(sizeof(int32_t) * (R / kRowSpan + 1));
  b += align_up(sizeof(int32_t) * T) * 2;
  b += align_up(sizeof(int32_t) * T * kHitStride);
  b += align_up(sizeof(float2) * T * kHitStride);
  b += align_up(sizeof(int32_t) * T) * 4;
  b += align_up(sizeof(float) * T);
  b += align_up(sizeof(float) * T * 6);
  b += align_up(sizeof(unsigned long long) * T);
  b += align_up(sizeof(int32_t) * T) * 4;
  b += align_up(sizeof(int32_t) * (2 * ((T + kSpan - 1) / kSpan) + 2));
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
  sc->g_rec = (GridRec*)take(sizeof(GridRec) * N);
  sc->up = (int32_t*)take(sizeof(int32_t) * N);
  sc->dn = (int32_t*)take(sizeof(int32_t) * N);
  sc->up2 = (int32_t*)take(sizeof(int32_t) * N);
  sc->dn2 = (int32_t*)take(sizeof(int32_t) * N);
  sc->start = (uint8_t*)take(sizeof(int32_t) * N);
  sc->own = (unsigned long long*)take(sizeof(unsigned long long) * N);
  sc->row_cnt = (int32_t*)take(sizeof(int32_t) * (R + 1));
  sc->row_part = (int32_t*)take(sizeof(int32_t) * (R / kRowSpan + 1));
  sc->cap_tl = (int32_t)T;
  sc->seeds = (int32_t*)take(sizeof(int32_t) * T);
  sc->seed_rs = (int32_t*)take(sizeof(int32_t) * T);
  sc->hits = (int32_t*)take(sizeof(int32_t) * T * kHitStride);
  sc->hit_yz = (float2*)take(sizeof(float2) * T * kHitStride);
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
  sc->span_sum = (int32_t*)take(sizeof(int32_t) * (2 * ((T + kSpan - 1) / kSpan) + 2));
  sc->ends = nullptr;
}

size_t global_bytes(int64_t N, int64_t T) {
  const int64_t Q = 2 * T;
  size_t b = 0;
  b += align_up(sizeof(float) * Q * kEndStride);
  b += align_up(sizeof(int32_t) * C_COUNT);
  b += align_up(sizeof(int32_t) * kLayoutSectors);
  b += align_up(sizeof(int32_t) * (N > 0 ? N : 1));
  b += align_up(sizeof(int32_t) * Q) * 2;
  b += align_up(sizeof(float) * Q * 8);
  b += align_up(sizeof(int32_t) * Q * kHitStride);
  b += align_up(sizeof(int32_t) * Q) * 5;
  b += align_up(sizeof(int32_t) * (2 * ((Q + kSpan - 1) / kSpan) + 2));
  return b;
}

void global_carve(void* base, int64_t N, int64_t T, float** ends, GlobalScratch* gs) {
  const int64_t Q = 2 * T;
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align_up(bytes);
    return r;
  };
  *ends = (float*)take(sizeof(float) * Q * kEndStride);
  gs->counters = (int32_t*)take(sizeof(int32_t) * C_COUNT);
  gs->p2s = (int32_t*)take(sizeof(int32_t) * kLayoutSectors);
  gs->claim = (int32_t*)take(sizeof(int32_t) * (N > 0 ? N : 1));
  gs->n = (int32_t*)take(sizeof(int32_t) * Q);
  gs->nslot = (int32_t*)take(sizeof(int32_t) * Q);
  gs->par = (float*)take(sizeof(float) * Q * 8);
  gs->hit = (int32_t*)take(sizeof(int32_t) * Q * kHitStride);
  gs->act = (int32_t*)take(sizeof(int32_t) * Q);
  gs->owned = (int32_t*)take(sizeof(int32_t) * Q);
  gs->kept = (int32_t*)take(sizeof(int32_t) * Q);
  gs->idx = (int32_t*)take(sizeof(int32_t) * Q);
  gs->off = (int32_t*)take(sizeof(int32_t) * Q);
  gs->span_sum = (int32_t*)take(sizeof(int32_t) * (2 * ((Q + kSpan - 1) / kSpan) + 2));
}

// Constructor: one lane per tracklet of the reservation, refills from the
// queue when the reservation exceeds the launch.  The launch covers up to 16
// million tracklets at 64 lanes: lanes that refill keep their waves alive
// with lanes in different phases, and a batch of 16 stress events spent 1.6
// times as long in the constructor with 16384 workgroups launched and the
// rest of its tracklets refilled.  Per-tracklet kernels: one wave per
// tracklet.
static inline int tl_blocks(int64_t T, int lanes) {
  int64_t b = (T + lanes - 1) / lanes;
  if (b > 262144) b = 262144;
  return (int)(b < 1 ? 1 : b);
}
// Both constructors give the tracklets of the sectors s = g (mod G) to the
// workgroups b = g (mod G), G <= 8: every group needs a workgroup, so the
// grid is a non-zero multiple of 8.
static inline int xcd_grid(int64_t b) {
  b = (b + 7) / 8 * 8;
  if (b < 8) b = 8;
  if (b > (int64_t)1 << 20) b = (int64_t)1 << 20;
  return (int)b;
}
// Row-synchronous constructor: workgroups loop over (sector, 64-tracklet
// chunk) items of their XCD group, so any grid is correct; this one gives
// every item a workgroup when the groups are not more than 25% uneven.
static inline int rows_blocks(int64_t T, int n_sectors) {
  int64_t per_group = (T + 511) / 512 * 5 / 4 + (n_sectors + 7) / 8 + 1;
  int64_t b = 8 * per_group;
  if (b > 65536) b = 65536;
  return (int)b;
}
static inline int wave_blocks(int64_t T) {
  int64_t b = (T + kGridBlock / 64 - 1) / (kGridBlock / 64);
  if (b > 65536) b = 65536;
  return (int)(b < 1 ? 1 : b);
}

const char* const kKernelNames[K_NUM] = {
    "k_zero", "k_grid", "k_nf", "k_evo", "k_scan_rows", "k_seed_write", "k_construct",
    "k_own", "k_tl_reduce", "k_tl_scan", "k_output", "k_pro_init", "k_ends", "k_prolong",
    "k_pro_own", "k_pro_reduce", "k_pro_scan", "k_pro_output", "k_mrg_init", "k_mrg_match",
    "k_mrg_link", "k_mrg_chain", "k_mrg_reduce", "k_mrg_scan", "k_mrg_write", "k_rowmap",
    "k_refit_gather", "k_refit"};

hipError_t enqueue_event(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const Outputs& out, int upto, hipStream_t st, const KernelTimer* tm,
                         bool zero_counters) {
  const int R = ev.n_sectors * kp.n_rows;
  auto pre = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][0], st);
  };
  auto post = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][1], st);
  };
  pre(K_ZERO);
  if (zero_counters) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, sc.counters);
  post(K_ZERO);
  pre(K_GRID);
  if (kp.row_wave)
    hipLaunchKernelGGL((k_grid<64, kGridWaveBins>), dim3(R), dim3(64), 0, st, ev, kp, sc,
                       out.cluster_track);
  else
    hipLaunchKernelGGL((k_grid<kGridBlock, kMaxBins>), dim3(R), dim3(kGridBlock), 0, st, ev, kp,
                       sc, out.cluster_track);
  post(K_GRID);
  if (upto <= STAGE_GRID) return hipGetLastError();
  pre(K_NF);
  if (kp.nf_stage == 2)
    hipLaunchKernelGGL((k_nf<kNfCapLarge, kNfListLarge, uint8_t, kNfDenseBlock>), dim3(R),
                       dim3(kNfDenseBlock), 0, st, ev, kp, sc);
  else if (kp.nf_stage == 3)
    hipLaunchKernelGGL((k_nf<kNfCapWave, kNfListSmall, uint16_t, 64>), dim3(R), dim3(64), 0, st,
                       ev, kp, sc);
  else
    hipLaunchKernelGGL((k_nf<kNfCapSmall, kNfListSmall, uint16_t, kGridBlock>), dim3(R),
                       dim3(kGridBlock), 0, st, ev, kp, sc);
  post(K_NF);
  pre(K_EVO);
  if (kp.row_wave)
    hipLaunchKernelGGL(k_evo<64>, dim3(R), dim3(64), 0, st, ev, kp, sc);
  else
    hipLaunchKernelGGL(k_evo<kGridBlock>, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc);
  post(K_EVO);
  if (upto <= STAGE_LINKS) return hipGetLastError();
  pre(K_SCAN_ROWS);
  {
    const int spans = max(1, (R + kRowSpan - 1) / kRowSpan);
    if (spans > 1) hipLaunchKernelGGL(k_rows_reduce, dim3(spans), dim3(kScanBlock), 0, st, R, sc);
    hipLaunchKernelGGL(k_scan_rows, dim3(spans), dim3(kScanBlock), 0, st, R, sc);
  }
  post(K_SCAN_ROWS);
  pre(K_SEED_WRITE);
  if (kp.row_wave)
    hipLaunchKernelGGL(k_seed_write<64>, dim3(R), dim3(64), 0, st, ev, sc);
  else
    hipLaunchKernelGGL(k_seed_write<kGridBlock>, dim3(R), dim3(kGridBlock), 0, st, ev, sc);
  post(K_SEED_WRITE);
  if (upto <= STAGE_SEEDS) return hipGetLastError();
  pre(K_CONSTRUCT);
  if (kp.construct_schedule == 1) {
    const int nb = xcd_grid(kp.construct_blocks > 0 ? kp.construct_blocks
                                                    : rows_blocks(sc.cap_tl, ev.n_sectors));
    if (sc.ends)
      hipLaunchKernelGGL(k_construct_rows<true>, dim3(nb), dim3(64), 0, st, ev, kp, sc);
    else
      hipLaunchKernelGGL(k_construct_rows<false>, dim3(nb), dim3(64), 0, st, ev, kp, sc);
  } else {
    const int A = min(max(kp.construct_lanes, 1), kTlBlock);
    const int nb = xcd_grid(kp.construct_blocks > 0 ? kp.construct_blocks : tl_blocks(sc.cap_tl, A));
    // the lanes' row slots in LDS when every wave that will get tracklets
    // (as many as the last call found per cluster) stays resident with them:
    // their LDS must not make waves wait for others to finish (waves beyond
    // the tracklets end at once); otherwise the hits array holds them
    const size_t lds = sizeof(int32_t) * kHitStride * A;
    int per_cu = 0;
    const hipError_t oe =
        sc.ends ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, k_construct_lanes<true, true>, kTlBlock, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, k_construct_lanes<false, true>, kTlBlock, lds);
    if (oe != hipSuccess) {
      (void)hipGetLastError();
      per_cu = 0;
    }
    const int64_t busy = ((int64_t)kp.expect_tl + A - 1) / A + 8;
    if (busy <= (int64_t)per_cu * kp.n_cu) {
      if (sc.ends)
        hipLaunchKernelGGL((k_construct_lanes<true, true>), dim3(nb), dim3(kTlBlock), lds, st, ev,
                           kp, sc);
      else
        hipLaunchKernelGGL((k_construct_lanes<false, true>), dim3(nb), dim3(kTlBlock), lds, st, ev,
                           kp, sc);
    } else {
      if (sc.ends)
        hipLaunchKernelGGL((k_construct_lanes<true, false>), dim3(nb), dim3(kTlBlock), 0, st, ev,
                           kp, sc);
      else
        hipLaunchKernelGGL((k_construct_lanes<false, false>), dim3(nb), dim3(kTlBlock), 0, st, ev,
                           kp, sc);
    }
  }
  post(K_CONSTRUCT);
  if (upto <= STAGE_TRACKLETS) return hipGetLastError();
  const int wb = wave_blocks(sc.cap_tl);
  pre(K_OWN);
  if (kp.own_by_sector)
    hipLaunchKernelGGL(k_own, dim3(ev.n_sectors * kOwnSplit), dim3(kOwnBlock), 0, st, ev, kp, sc);
  else
    hipLaunchKernelGGL(k_own, dim3(ev.n_sectors, kOwnSplit), dim3(kOwnBlock), 0, st, ev, kp, sc);
  post(K_OWN);
  const int spans = (int)((sc.cap_tl + kSpan - 1) / kSpan);
  pre(K_TL_REDUCE);
  hipLaunchKernelGGL(k_tl_reduce, dim3(spans), dim3(kScanBlock), 0, st, sc, kp.min_clusters);
  post(K_TL_REDUCE);
  pre(K_TL_SCAN);
  hipLaunchKernelGGL(k_tl_scan, dim3(spans), dim3(kScanBlock), 0, st, sc, kp.min_clusters,
                     out.cap_tracks, out.cap_track_clusters);
  post(K_TL_SCAN);
  pre(K_OUTPUT);
  hipLaunchKernelGGL(k_output, dim3(wb), dim3(kGridBlock), 0, st, ev, kp, sc, out);
  post(K_OUTPUT);
  return hipGetLastError();
}

hipError_t enqueue_global(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                          const Outputs& out, const GlobalScratch& gs, const ProOutputs* po,
                          hipStream_t st, const KernelTimer* tm, int part) {
  auto pre = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][0], st);
  };
  auto post = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][1], st);
  };
  const int64_t Q = 2 * (int64_t)sc.cap_tl;
  const int cb = (int)std::min<int64_t>(std::max<int64_t>((ev.n_clusters + kGridBlock - 1) /
                                                              kGridBlock, 1), 2048);
  const int qb = (int)std::min<int64_t>(std::max<int64_t>((Q + kGridBlock - 1) / kGridBlock, 1),
                                        65535);
  if (part != 1) {
    pre(K_PRO_INIT);
    hipLaunchKernelGGL(k_pro_init, dim3(cb), dim3(kGridBlock), 0, st, ev, kp, sc, gs,
                       po ? (const int32_t*)out.cluster_track : nullptr);
    post(K_PRO_INIT);
    pre(K_ENDS);
    hipLaunchKernelGGL(k_ends, dim3(qb), dim3(kGridBlock), 0, st, kp, sc, gs);
    post(K_ENDS);
  }
  if (!po || part == 0) return hipGetLastError();
  pre(K_PROLONG);
  hipLaunchKernelGGL(k_prolong, dim3(qb), dim3(kGridBlock), 0, st, ev, kp, sc, gs);
  post(K_PROLONG);
  pre(K_PRO_OWN);
  hipLaunchKernelGGL(k_pro_own, dim3(qb), dim3(kGridBlock), 0, st, sc, gs);
  post(K_PRO_OWN);
  // numbering of the slots that own clusters: the selection's scan over slots
  Scratch ps = sc;
  ps.counters = gs.counters;
  ps.cap_tl = (int32_t)Q;
  ps.owned = gs.owned;
  ps.kept = gs.kept;
  ps.trk_idx = gs.idx;
  ps.trk_off = gs.off;
  ps.span_sum = gs.span_sum;
  const int spans = (int)((Q + kSpan - 1) / kSpan);
  pre(K_PRO_REDUCE);
  hipLaunchKernelGGL(k_tl_reduce, dim3(spans), dim3(kScanBlock), 0, st, ps, 1);
  post(K_PRO_REDUCE);
  pre(K_PRO_SCAN);
  hipLaunchKernelGGL(k_tl_scan, dim3(spans), dim3(kScanBlock), 0, st, ps, 1, po->cap,
                     po->cap_clusters);
  post(K_PRO_SCAN);
  pre(K_PRO_OUTPUT);
  hipLaunchKernelGGL(k_pro_output, dim3(wave_blocks(Q)), dim3(kGridBlock), 0, st, ev, sc, gs,
                     *po);
  post(K_PRO_OUTPUT);
  return hipGetLastError();
}

size_t merge_bytes(int64_t N, int64_t S, int64_t T, int64_t cap_rec) {
  size_t b = 0;
  b += align_up(sizeof(int32_t) * C_COUNT);
  b += align_up(sizeof(int32_t) * (S + 1));
  b += align_up(sizeof(float4) * 2 * T);
  b += align_up(sizeof(int32_t) * T) * 2;
  b += align_up(sizeof(unsigned long long) * T);
  b += align_up(sizeof(int32_t) * T) * 6;
  b += align_up(sizeof(int32_t) * (2 * ((T + kSpan - 1) / kSpan) + 2));
  b += align_up(sizeof(int32_t) * (T + 1));
  b += align_up(sizeof(int32_t) * (N > 0 ? N : 1));
  b += align_up(sizeof(float4) * (cap_rec > 0 ? cap_rec : 1));
  return b;
}

void merge_carve(void* base, int64_t N, int64_t S, int64_t T, int64_t cap_rec,
                 MergeScratch* ms) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align_up(bytes);
    return r;
  };
  ms->counters = (int32_t*)take(sizeof(int32_t) * C_COUNT);
  ms->first = (int32_t*)take(sizeof(int32_t) * (S + 1));
  ms->sum = (float4*)take(sizeof(float4) * 2 * T);
  ms->next = (int32_t*)take(sizeof(int32_t) * T);
  ms->best = (int32_t*)take(sizeof(int32_t) * T);
  ms->prev_key = (unsigned long long*)take(sizeof(unsigned long long) * T);
  ms->prev = (int32_t*)take(sizeof(int32_t) * T);
  ms->cnt = (int32_t*)take(sizeof(int32_t) * T);
  ms->nseg = (int32_t*)take(sizeof(int32_t) * T);
  ms->kept = (int32_t*)take(sizeof(int32_t) * T);
  ms->idx = (int32_t*)take(sizeof(int32_t) * T);
  ms->off = (int32_t*)take(sizeof(int32_t) * T);
  ms->span_sum = (int32_t*)take(sizeof(int32_t) * (2 * ((T + kSpan - 1) / kSpan) + 2));
  ms->loff = (int32_t*)take(sizeof(int32_t) * (T + 1));
  ms->rowslot = (int32_t*)take(sizeof(int32_t) * (N > 0 ? N : 1));
  ms->rec = (float4*)take(sizeof(float4) * (cap_rec > 0 ? cap_rec : 1));
  ms->cap_rec = (int32_t)cap_rec;
}

hipError_t enqueue_merge(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const Outputs& out, const GlobalScratch& gs, const ProOutputs* po,
                         const MergeScratch& ms, const MergeOutputs& mo, hipStream_t st,
                         const KernelTimer* tm, int part) {
  auto pre = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][0], st);
  };
  auto post = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][1], st);
  };
  const int64_t T = sc.cap_tl;
  const int tb = (int)std::min<int64_t>(std::max<int64_t>((T + kGridBlock - 1) / kGridBlock, 1),
                                        65535);
  const int R = ev.n_sectors * kp.n_rows;
  if (part != 1) {  // the joins need only the end states (and the event)
    pre(K_MRG_INIT);
    hipLaunchKernelGGL(k_mrg_init, dim3(tb), dim3(kGridBlock), 0, st, ev, kp, sc, gs, ms);
    post(K_MRG_INIT);
    pre(K_MRG_MATCH);
    hipLaunchKernelGGL(k_mrg_match, dim3(wave_blocks(T)), dim3(kGridBlock), 0, st, ev, kp, sc,
                       gs, ms);
    post(K_MRG_MATCH);
    pre(K_MRG_LINK);
    hipLaunchKernelGGL(k_mrg_link, dim3(tb), dim3(kGridBlock), 0, st, sc, ms);
    post(K_MRG_LINK);
    pre(K_ROWMAP);
    hipLaunchKernelGGL(k_rowmap, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc, ms);
    post(K_ROWMAP);
  }
  if (part == 0) return hipGetLastError();
  // the chains' lists need the prolongations
  pre(K_MRG_CHAIN);
  hipLaunchKernelGGL(k_mrg_chain, dim3(tb), dim3(kGridBlock), 0, st, sc, gs, ms, out,
                     po ? 1 : 0);
  post(K_MRG_CHAIN);
  // numbering of the chains: the selection's scan over tracks
  Scratch ps = sc;
  ps.counters = ms.counters;
  ps.owned = ms.cnt;
  ps.kept = ms.kept;
  ps.trk_idx = ms.idx;
  ps.trk_off = ms.off;
  ps.span_sum = ms.span_sum;
  const int spans = (int)((T + kSpan - 1) / kSpan);
  pre(K_MRG_REDUCE);
  hipLaunchKernelGGL(k_tl_reduce, dim3(spans), dim3(kScanBlock), 0, st, ps, 1);
  post(K_MRG_REDUCE);
  pre(K_MRG_SCAN);
  hipLaunchKernelGGL(k_tl_scan, dim3(spans), dim3(kScanBlock), 0, st, ps, 1, mo.cap,
                     mo.cap_clusters);
  post(K_MRG_SCAN);
  const ProOutputs pz{0, 0, nullptr, nullptr, nullptr};
  pre(K_MRG_WRITE);
  hipLaunchKernelGGL(k_mrg_write, dim3(wave_blocks(T)), dim3(kGridBlock), 0, st, ev, kp, sc, gs,
                     ms, out, po ? *po : pz, po ? 1 : 0, mo);
  post(K_MRG_WRITE);
  pre(K_REFIT_GATHER);
  const int gb = (int)std::min<int64_t>(std::max<int64_t>((ms.cap_rec + kGridBlock - 1) /
                                                              kGridBlock, 1), 4096);
  hipLaunchKernelGGL(k_refit_gather, dim3(gb), dim3(kGridBlock), 0, st, ev, kp.n_rows, sc, ms,
                     (const int32_t*)&ms.counters[C_TRACK_CLUSTERS], 0,
                     (const int32_t*)mo.cluster);
  post(K_REFIT_GATHER);
  pre(K_REFIT);
  hipLaunchKernelGGL(k_refit, dim3(tb), dim3(kGridBlock), 0, st, ev, kp, sc, ms,
                     (const int32_t*)&ms.counters[C_TRACKS], 0, ms.cap_rec,
                     (const int32_t*)ms.loff, mo.par, (int32_t*)nullptr, mo.meta);
  post(K_REFIT);
  return hipGetLastError();
}

hipError_t enqueue_refit(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const MergeScratch& ms, int32_t n_lists, int32_t n_entries,
                         const int32_t* offsets, const int32_t* clusters, float* par,
                         int32_t* frame, hipStream_t st, const KernelTimer* tm) {
  auto pre = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][0], st);
  };
  auto post = [&](int k) {
    if (tm && (tm->mask >> k & 1u)) (void)hipEventRecord(tm->ev[k][1], st);
  };
  const int R = ev.n_sectors * kp.n_rows;
  pre(K_ROWMAP);
  hipLaunchKernelGGL(k_rowmap, dim3(R), dim3(kGridBlock), 0, st, ev, kp, sc, ms);
  post(K_ROWMAP);
  if (n_lists > 0) {
    if (n_entries > 0) {
      const int gb = std::min((n_entries + kGridBlock - 1) / kGridBlock, 4096);
      pre(K_REFIT_GATHER);
      hipLaunchKernelGGL(k_refit_gather, dim3(gb), dim3(kGridBlock), 0, st, ev, kp.n_rows, sc,
                         ms, (const int32_t*)nullptr, n_entries, clusters);
      post(K_REFIT_GATHER);
    }
    const int lb = std::min((n_lists + kGridBlock - 1) / kGridBlock, 65535);
    pre(K_REFIT);
    hipLaunchKernelGGL(k_refit, dim3(lb), dim3(kGridBlock), 0, st, ev, kp, sc, ms,
                       (const int32_t*)nullptr, n_lists, n_entries, offsets, par, frame,
                       (int32_t*)nullptr);
    post(K_REFIT);
  }
  return hipGetLastError();
}

}  // namespace tpc
