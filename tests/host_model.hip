// Host build of the kernels' track model (tpc_model.h) for the CPU tests:
// a tracklet's fit replayed through the same FP32/FP64 arithmetic the
// constructor runs, given the clusters it collected.  Test infrastructure,
// compiled with hipcc --offload-host-only; no GPU is needed.
#include <string.h>

#include "../paper_1712_09407_amd/csrc/tpc_model.h"

namespace {

// prm: sy2, sz2, k_curv, bz, max_sinphi, prior_sinphi, prior_tanl, prior_qpt
tpc::KParams make_params(const float* prm) {
  tpc::KParams kp{};
  kp.sy2 = prm[0];
  kp.sz2 = prm[1];
  kp.k_curv = prm[2];
  kp.bz = prm[3];
  kp.max_sinphi = prm[4];
  kp.prior_sinphi = prm[5];
  kp.prior_tanl = prm[6];
  kp.prior_qpt = prm[7];
  return kp;
}

}  // namespace

extern "C" {

// The constructor's fit of one tracklet whose clusters are known: the seed
// circle through rows k0, k0 + ms/2 and k0 + ms - 1, the outward filter from
// row k0 + 1 to row hi (a helix step on every row, an update on every row
// with a cluster), then the inward fit from the cluster of row hi with a
// fresh covariance down to row lo.  has[r], hy[r], hz[r]: the cluster of row
// r.  out: x, y, z, sin phi, tan lambda, q/pT at the innermost cluster, chi^2
// of the inward fit, then the outward state at row hi (sin phi, tan lambda,
// q/pT).  Returns the number of clusters of the inward fit, or -1 if a step
// failed.
int host_fit_tracklet(const float* row_x, const int* has, const float* hy, const float* hz,
                      int lo, int hi, int k0, int ms, const float* prm, float* out) {
  const tpc::KParams kp = make_params(prm);
  const int b = k0 + ms / 2, e = k0 + ms - 1;
  tpc::KState s;
  tpc::seed3(s, row_x[k0], hy[k0], hz[k0], row_x[b], hy[b], row_x[e], hy[e], hz[e], kp);
  if (fabsf(s.sp) > kp.max_sinphi) return -1;
  for (int r = k0 + 1; r <= hi; ++r) {
    if (!tpc::propagate(s, row_x[r], kp)) return -1;
    if (has[r]) tpc::kf_update(s, hy[r], hz[r], kp);
  }
  out[7] = s.sp;
  out[8] = s.tl;
  out[9] = s.qpt;
  tpc::KState w;
  w.x = row_x[hi];
  w.y = hy[hi];
  w.z = hz[hi];
  w.sp = s.sp;
  w.tl = s.tl;
  w.qpt = s.qpt;
  tpc::reset_cov(w.C, kp);
  float chi2 = 0.f;
  int n = 1;
  float o[6] = {w.x, w.y, w.z, w.sp, w.tl, w.qpt};
  for (int r = hi - 1; r >= lo; --r) {
    if (!tpc::propagate(w, row_x[r], kp)) return -1;
    if (has[r]) {
      chi2 += tpc::kf_update(w, hy[r], hz[r], kp);
      ++n;
      o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.sp; o[4] = w.tl; o[5] = w.qpt;
    }
  }
  for (int i = 0; i < 6; ++i) out[i] = o[i];
  out[6] = chi2;
  return n;
}

// One helix step of a state with its covariance (packed lower triangle,
// 15 values): the kernels' propagate.  Returns 0, or 1 if it stopped.
int host_propagate(float* state /* x, y, z, sp, tl, qpt */, double* cov, float x2,
                   const float* prm) {
  const tpc::KParams kp = make_params(prm);
  tpc::KState s;
  s.x = state[0]; s.y = state[1]; s.z = state[2]; s.sp = state[3]; s.tl = state[4];
  s.qpt = state[5];
  memcpy(&s.C, cov, sizeof(tpc::Cov));
  if (!tpc::propagate(s, x2, kp)) return 1;
  state[0] = s.x; state[1] = s.y; state[2] = s.z; state[3] = s.sp; state[4] = s.tl;
  state[5] = s.qpt;
  memcpy(cov, &s.C, sizeof(tpc::Cov));
  return 0;
}

}  // extern "C"
