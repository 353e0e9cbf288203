// Pooled projection: the body shared by the library's projection kernel and
// the kernels compiled at run time for one robot and constraint mask.
#pragma once
#include "device.h"
#include "project.h"

namespace cprrtc {

// Pooled projection (modes 0-2): one wavefront keeps S motions in LDS and,
// every iteration, spreads only their active waypoints (k > prog) over its 64
// lanes in rounds of 64, so no lane spends an iteration on a frozen prefix.
// Item i of an iteration is waypoint prog_s + 1 + (i - off_s) of slot s
// (off = prefix sums of the slots' active counts).  Each item reads its
// waypoint and the previous one from the slot's snapshot in LDS and computes
// the same update as project_segment.  A slot's new prog is the number of
// leading valid items (first invalid item from the rounds' ballots); items
// past it take their new values, written as soon as their round is judged
// (the one waypoint a later round still reads from the snapshot is carried
// over in registers).  A finished motion (success, or failure
// after max_iters) is written out and its slot refilled from the
// wavefront's share of the motions (a contiguous run).
// The body is a device function so that the kernel compiled with the
// library (policy RobotMem) and kernels compiled at run time for one robot
// and constraint mask (a constant policy) share it.  One wavefront per
// workgroup (64 lanes).
template <int NDOF, int KIND, int MODE, int S, class P>
__device__ __forceinline__ void project_pool_body(
    const RobotDev* __restrict__ rob, const ConDev& con, const ProjDev& prm, int n_motions,
    const float* __restrict__ q_from, const float* __restrict__ q_to,
    const float* __restrict__ delta, float* __restrict__ xi, int* __restrict__ status,
    int* __restrict__ iters, unsigned long long* __restrict__ work) {
  __shared__ float sx[S][64][NDOF];
  const int lane = threadIdx.x;
  const int W = prm.W;
  // this wavefront's share: a contiguous run of motions, so that the
  // wavefronts of a neighbourhood read and write neighbouring lines
  const int chunk = (n_motions + (int)gridDim.x - 1) / (int)gridDim.x;
  int next = (int)blockIdx.x * chunk;    // wavefront-uniform local queue
  const int share_end = min(next + chunk, n_motions);
  int mot[S], prog[S], its[S];
  unsigned long long updates = 0;

  // Fills slot s with the wavefront's next motion (straight-line segment,
  // plus the network's correction in MODE 1); mot[s] = -1 when none is left.
  auto fetch = [&](int s) {
    int m = -1;
    while (next < share_end) {
      const int cand = next;
      ++next;
      if (MODE != 2 || status[cand] == 1) {
        m = cand;
        break;
      }
    }
    mot[s] = m;
    prog[s] = 0;
    its[s] = 0;
    if (m >= 0 && lane < W) {
      const float t = (float)lane / (float)(W - 1);
#pragma unroll
      for (int j = 0; j < NDOF; ++j) {
        const float a = q_from[(int64_t)m * NDOF + j];
        const float b = q_to[(int64_t)m * NDOF + j];
        float v = a + t * (b - a);
        if (MODE == 1 && lane >= 1)
          v = fminf(fmaxf(v + delta[((int64_t)m * (W - 1) + (lane - 1)) * NDOF + j], P::lo(rob, j)),
                    P::hi(rob, j));
        sx[s][lane][j] = v;
      }
    }
  };

#pragma unroll
  for (int s = 0; s < S; ++s) fetch(s);
  __syncthreads();

  while (true) {
    int off[S + 1];
    off[0] = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) off[s + 1] = off[s] + (mot[s] >= 0 ? W - 1 - prog[s] : 0);
    const int A = off[S];
    if (A == 0) break;                   // every slot empty: the share is done
    updates += (unsigned long long)A;

    int first_bad[S];
#pragma unroll
    for (int s = 0; s < S; ++s) first_bad[s] = W;
    float carry[NDOF];                   // snapshot of the previous round's last item
#pragma unroll
    for (int j = 0; j < NDOF; ++j) carry[j] = 0.0f;
    for (int base = 0; base < A; base += 64) {   // uniform trip count
      const int i = base + lane;
      const bool on = i < A;
      int si = 0, sp = prog[0], so = off[0];
#pragma unroll
      for (int s = 1; s < S; ++s)
        if (i >= off[s]) { si = s; sp = prog[s]; so = off[s]; }
      const int k = on ? sp + 1 + (i - so) : 1;
      // Items are consecutive waypoints of their slot, so only the first
      // lane can need a waypoint that the previous round already moved: it
      // takes that round's snapshot value (carry) instead.
      const bool from_carry = lane == 0 && base > 0 && i - 1 >= so;
      float q[NDOF], qp[NDOF], qn[NDOF];
#pragma unroll
      for (int j = 0; j < NDOF; ++j) {
        q[j] = sx[si][k][j];
        qp[j] = from_carry ? carry[j] : sx[si][k - 1][j];
      }
      bool valid = true;
      if (on) valid = waypoint_update<NDOF, KIND, P>(rob, con, prm, q, qp, qn);
      const uint64_t inv = __ballot(on && !valid);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int lo = max(off[s] - base, 0), hi = min(off[s + 1] - base, 64);
        if (lo < hi && first_bad[s] == W) {
          const uint64_t span = (hi - lo == 64) ? ~0ull : (((1ull << (hi - lo)) - 1ull) << lo);
          const uint64_t m = inv & span;
          if (m) first_bad[s] = base + (__ffsll((unsigned long long)m) - 1) - off[s];
        }
      }
#pragma unroll
      for (int j = 0; j < NDOF; ++j) carry[j] = __shfl(q[j], 63, 64);
      // Every item before this one in its slot has been judged: it moves
      // iff an invalid item precedes it or is it (it lies past the new prog).
      int fb = first_bad[0];
#pragma unroll
      for (int s = 1; s < S; ++s)
        if (si == s) fb = first_bad[s];
      if (on && i - so >= fb) {
#pragma unroll
        for (int j = 0; j < NDOF; ++j) sx[si][k][j] = qn[j];
      }
    }
    int newprog[S];
#pragma unroll
    for (int s = 0; s < S; ++s) newprog[s] = prog[s] + min(first_bad[s], W - 1 - prog[s]);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (mot[s] < 0) continue;
      its[s] += 1;
      prog[s] = newprog[s];
      const bool ok = prog[s] == W - 1;
      if (!ok && its[s] < prm.max_iters) continue;
      const int m = mot[s];
      if (lane < W) {
#pragma unroll
        for (int j = 0; j < NDOF; ++j) xi[((int64_t)m * W + lane) * NDOF + j] = sx[s][lane][j];
      }
      if (lane == 0) {
        status[m] = ok ? 0 : 1;
        if (iters) iters[m] = (MODE == 2 ? iters[m] : 0) + (ok ? its[s] : prm.max_iters);
      }
      __syncthreads();                   // the slot is read out before it is refilled
      fetch(s);
    }
    __syncthreads();
  }
  if (work && lane == 0) atomicAdd(&work[6], updates);
}

}  // namespace cprrtc
