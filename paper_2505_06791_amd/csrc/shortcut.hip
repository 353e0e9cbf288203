// Path shortcutting: rounds of batched shortcut motions over a dense path.
// The candidates of a round are projected and validated together by the
// library's own motion kernels (one call of project_validate_motions); the
// choice of candidates and the splicing of accepted pieces run on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cprrtc.h"
#include "handles.h"

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

double dist(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += (a[j] - b[j]) * (a[j] - b[j]);
  return std::sqrt(s);
}

struct Piece {
  int i, j;
  double gain;
  int slot;   // candidate index (row of xi)
};

}  // namespace

extern "C" {

int cp_shortcut(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
                const cp_proj_params* params, const double* path, int32_t len, int32_t rounds,
                int32_t flags, cp_path* out, cp_shortcut_stats* stats, void* stream) {
  using namespace cprrtc;
  try {
    if (!robot || !env || !path || !out) return api_fail(CP_E_ARG, "cp_shortcut: NULL argument");
    if (len < 1 || rounds < 0) return api_fail(CP_E_ARG, "cp_shortcut: len < 1 or rounds < 0");
    if (flags & ~(CP_NO_EARLY_EXIT | CP_NO_CULL | CP_POOLED | CP_PER_MOTION | CP_GENERIC |
                  CP_SELF_COLLISION))
      return api_fail(CP_E_ARG, "cp_shortcut: unknown flags %d", flags);
    cp_proj_params p;
    cp_proj_params_default(&p);
    if (params) p = *params;
    const int n = robot->host.dof, W = p.W;
    if (W != 32 && W != 64) return api_fail(CP_E_UNSUPPORTED, "cp_shortcut: W = %d", W);
    const double reach = (W - 1) * p.tau;          // the steer length
    const double link = p.tau + p.tau_sm;          // largest valid spacing
    std::vector<double> P(path, path + (size_t)len * n);
    hipStream_t st = (hipStream_t)stream;
    cp_shortcut_stats s;
    std::memset(&s, 0, sizeof s);
    auto length = [&](const std::vector<double>& v) {
      double t = 0.0;
      for (size_t k = 1; k < v.size() / n; ++k) t += dist(&v[(k - 1) * n], &v[k * n], n);
      return t;
    };
    s.length_before = length(P);
    DevBuf qf, qt, xi, status;
    int cap = 0;
    for (int r = 0; r < rounds; ++r) {
      const int L = (int)(P.size() / n);
      // candidates: for each i, the farthest j >= i + 2 within the steer
      // length, if the subpath between them is longer than the chord
      std::vector<int> ci, cj;
      for (int i = 0; i + 2 < L; ++i) {
        int j = -1;
        for (int k = L - 1; k >= i + 2; --k)
          if (dist(&P[(size_t)i * n], &P[(size_t)k * n], n) <= reach) {
            j = k;
            break;
          }
        if (j < 0) continue;
        double sub = 0.0;
        for (int k = i; k < j; ++k) sub += dist(&P[(size_t)k * n], &P[(size_t)(k + 1) * n], n);
        if (sub - dist(&P[(size_t)i * n], &P[(size_t)j * n], n) <= 1e-9) continue;
        ci.push_back(i);
        cj.push_back(j);
      }
      const int M = (int)ci.size();
      if (M == 0) break;
      if (M > cap) {
        for (DevBuf* b : {&qf, &qt, &xi, &status}) {
          if (b->p) (void)hipFree(b->p);
          b->p = nullptr;
        }
        hipError_t e = hipMalloc(&qf.p, sizeof(float) * (size_t)M * n);
        if (e == hipSuccess) e = hipMalloc(&qt.p, sizeof(float) * (size_t)M * n);
        if (e == hipSuccess) e = hipMalloc(&xi.p, sizeof(float) * (size_t)M * W * n);
        if (e == hipSuccess) e = hipMalloc(&status.p, sizeof(int32_t) * (size_t)M);
        if (e != hipSuccess) return api_hip_fail(e, "cp_shortcut buffers");
        cap = M;
      }
      std::vector<float> hf((size_t)M * n), ht((size_t)M * n);
      for (int m = 0; m < M; ++m)
        for (int jj = 0; jj < n; ++jj) {
          hf[(size_t)m * n + jj] = (float)P[(size_t)ci[m] * n + jj];
          ht[(size_t)m * n + jj] = (float)P[(size_t)cj[m] * n + jj];
        }
      hipError_t e = hipMemcpyAsync(qf.p, hf.data(), sizeof(float) * hf.size(),
                                    hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(qt.p, ht.data(), sizeof(float) * ht.size(), hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return api_hip_fail(e, "cp_shortcut upload");
      int rc = project_validate_motions(robot, env, constraint, &p, M, (const float*)qf.p,
                                        (const float*)qt.p, (float*)xi.p, (int32_t*)status.p,
                                        nullptr, nullptr, flags, stream);
      if (rc != CP_OK) return rc;
      std::vector<float> hx((size_t)M * W * n);
      std::vector<int32_t> hs(M);
      e = hipMemcpyAsync(hx.data(), xi.p, sizeof(float) * hx.size(), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hs.data(), status.p, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return api_hip_fail(e, "cp_shortcut download");
      s.candidates += M;
      // accepted pieces: a valid motion whose last free waypoint but one
      // reaches P[j] within a valid spacing, shorter than the subpath; the
      // piece is waypoints 1 .. W-2, then P[j] itself
      std::vector<Piece> acc;
      std::vector<double> wp(n);
      for (int m = 0; m < M; ++m) {
        if (hs[m] != CP_MOTION_VALID) continue;
        const int i = ci[m], j = cj[m];
        const float* x = &hx[(size_t)m * W * n];
        for (int jj = 0; jj < n; ++jj) wp[jj] = (double)x[(size_t)(W - 2) * n + jj];
        if (!(dist(wp.data(), &P[(size_t)j * n], n) < link)) continue;
        double piece = 0.0;
        std::vector<double> prev(&P[(size_t)i * n], &P[(size_t)i * n] + n), cur(n);
        for (int k = 1; k <= W - 2; ++k) {
          for (int jj = 0; jj < n; ++jj) cur[jj] = (double)x[(size_t)k * n + jj];
          piece += dist(prev.data(), cur.data(), n);
          prev.swap(cur);
        }
        piece += dist(prev.data(), &P[(size_t)j * n], n);
        double sub = 0.0;
        for (int k = i; k < j; ++k) sub += dist(&P[(size_t)k * n], &P[(size_t)(k + 1) * n], n);
        if (piece < sub) acc.push_back({i, j, sub - piece, m});
      }
      if (acc.empty()) {
        s.rounds = r + 1;
        break;
      }
      // largest gains first; a piece is kept if its interval [i, j] meets
      // no kept interval except at an end point
      std::stable_sort(acc.begin(), acc.end(),
                       [](const Piece& a, const Piece& b) { return a.gain > b.gain; });
      std::vector<Piece> keep;
      for (const Piece& c : acc) {
        bool ok = true;
        for (const Piece& k : keep)
          if (!(c.j <= k.i || k.j <= c.i)) ok = false;
        if (ok) keep.push_back(c);
      }
      std::sort(keep.begin(), keep.end(), [](const Piece& a, const Piece& b) { return a.i < b.i; });
      std::vector<double> Q;
      int at = 0;
      for (const Piece& c : keep) {
        Q.insert(Q.end(), P.begin() + (size_t)at * n, P.begin() + (size_t)(c.i + 1) * n);
        const float* x = &hx[(size_t)c.slot * W * n];
        for (int k = 1; k <= W - 2; ++k)
          for (int jj = 0; jj < n; ++jj) Q.push_back((double)x[(size_t)k * n + jj]);
        at = c.j;
      }
      Q.insert(Q.end(), P.begin() + (size_t)at * n, P.end());
      P.swap(Q);
      s.replaced += (int)keep.size();
      s.rounds = r + 1;
    }
    s.length_after = length(P);
    if (stats) *stats = s;
    out->dof = n;
    out->len = (int32_t)(P.size() / n);
    if (out->capacity < out->len || !out->q)
      return api_fail(CP_E_CAPACITY, "cp_shortcut: path of %d rows, capacity %d", out->len,
                      out->capacity);
    std::memcpy(out->q, P.data(), sizeof(double) * P.size());
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_shortcut: unexpected exception");
  }
}

}  // extern "C"
