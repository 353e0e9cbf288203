// Pooled projection: the body shared by the library's projection kernel and
// the kernels compiled at run time for one robot and constraint mask.
#pragma once
#include "device.h"
#include "project.h"

namespace cprrtc {

// The slot bookkeeping (motion ids, progress, offsets, first invalid item)
// is the same on every lane; keeping it in scalar registers takes it off the
// vector pipe, which the waypoint updates keep busy.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// This lane's bit of a wavefront-uniform mask.  Compilers that have the
// inverse ballot use the mask as the lane predicate directly; older ones
// (the run-time compiler may be one) shift and test it.
__device__ __forceinline__ bool lane_in(uint64_t mask) {
#if __has_builtin(__builtin_amdgcn_inverse_ballot_w64)
  return __builtin_amdgcn_inverse_ballot_w64(mask);
#else
  return (mask >> threadIdx.x) & 1ull;
#endif
}

// Lanes lo .. hi-1 of a wavefront as a mask (0 <= lo, hi <= 64).
__device__ __forceinline__ uint64_t lane_range(int lo, int hi) {
  if (lo >= hi) return 0;
  const uint64_t upto = hi >= 64 ? ~0ull : (1ull << hi) - 1ull;
  return upto & ~((1ull << lo) - 1ull);
}

// Pooled projection (modes 0-2): one wavefront keeps S motions in LDS and
// streams their active waypoints (k > prog) over its 64 lanes in rounds of
// 64 items, so no lane spends an iteration on a frozen prefix.  A slot's
// iteration is the run of items prog_s + 1 .. W - 1; rounds take the next
// items of the slots in ring order, each slot at most once per round, so a
// round may end one slot's iteration and begin or continue another's, and
// a slot's next iteration starts in a later round, after this one is judged.
// Each item reads its waypoint and the previous one from the slot's
// snapshot in LDS and computes the same update as project_segment.  A
// slot's new prog is the number of leading valid items (first invalid item
// from the rounds' ballots); items past it take their new values, written
// as soon as their round is judged (the one waypoint a later round still
// reads from the snapshot is kept aside in LDS).  A finished motion
// (success, or failure after max_iters) is written out and its slot
// refilled from the wavefront's share of the motions (a contiguous run).
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
  __shared__ float sprev[NDOF];        // the previous round's last snapshot
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
    mot[s] = uniform(m);
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

  // per slot, uniform: items of the current iteration (0: empty slot), items
  // already dispatched, first invalid item, row of item 0 in sx
  int cnt[S], pos[S], first_bad[S], kb[S];
  auto begin_iteration = [&](int s) {
    cnt[s] = mot[s] >= 0 ? W - 1 - prog[s] : 0;
    pos[s] = 0;
    first_bad[s] = W;
    kb[s] = uniform(s * 64 + prog[s] + 1);
  };
#pragma unroll
  for (int s = 0; s < S; ++s) {
    fetch(s);
    begin_iteration(s);
  }
  __syncthreads();

  float* const rows = &sx[0][0][0];
  int cursor = 0;                        // slot the next round starts with
  while (true) {
    // Fill the round's 64 lanes with the next items of the slots in ring
    // order from the cursor, each slot at most once (a slot's next iteration
    // waits for a later round, when its current one is judged and written).
    int off[S], n[S];
    int left = 64, next_cursor = cursor;
    bool full = false;
#pragma unroll
    for (int t = 0; t < 2 * S; ++t) {
      const int s = t % S;
      if (t < S) {
        off[s] = 0;
        n[s] = 0;
      }
      const bool turn = t < S ? s >= cursor : s < cursor;
      if (turn && !full && cnt[s] > 0) {
        const int rem = cnt[s] - pos[s];
        const int take = min(rem, left);
        off[s] = 64 - left;
        n[s] = take;
        left -= take;
        if (take < rem) {
          full = true;                   // slot s continues next round
          next_cursor = s;
        } else if (left == 0) {
          full = true;
          next_cursor = s + 1 == S ? 0 : s + 1;
        }
      }
    }
    if (left == 64) break;               // every slot empty: the share is done
    cursor = next_cursor;
    updates += (unsigned long long)(64 - left);

    uint64_t span[S];
    int row = 1;                         // lanes past the last item read a valid row
    bool carried = false;                // lane 0 continues a slot from the previous round
#pragma unroll
    for (int s = 0; s < S; ++s) {
      span[s] = lane_range(off[s], off[s] + n[s]);
      if (span[s] && lane_in(span[s])) row = lane + uniform(kb[s] + pos[s] - off[s]);
      carried = carried || (n[s] > 0 && off[s] == 0 && pos[s] > 0);
    }
    const bool on = lane < 64 - left;
    // Items are consecutive waypoints of their slot, so only the first lane
    // can need a waypoint that the previous round already moved: it reads
    // that round's snapshot of it (sprev) instead.
    const int at = __mul24(row, NDOF);   // row < S * 64
    const float* prev = (carried && lane == 0) ? sprev : rows + (at - NDOF);
    float q[NDOF], qp[NDOF], qn[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      q[j] = rows[at + j];
      qp[j] = prev[j];
    }
    bool valid = true;
    if (on) valid = waypoint_update<NDOF, KIND, P>(rob, con, prm, q, qp, qn);
    const uint64_t inv = uniform((uint64_t)__ballot(on && !valid));
    // Every item before this one in its slot has been judged: it moves iff
    // an invalid item precedes it or is it (it lies past the new prog).
    uint64_t moves = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (!span[s]) continue;
      const uint64_t m = inv & span[s];
      if (first_bad[s] == W && m)
        first_bad[s] = uniform(pos[s] + (__ffsll((unsigned long long)m) - 1) - off[s]);
      if (first_bad[s] < W)
        moves |= span[s] & ~lane_range(0, min(max(off[s] + first_bad[s] - pos[s], 0), 64));
    }
    // (one wavefront: its LDS accesses complete in program order, so this
    // store follows this round's reads and precedes the next round's)
    if (lane == 63) {
#pragma unroll
      for (int j = 0; j < NDOF; ++j) sprev[j] = q[j];
    }
    if (lane_in(moves)) {
#pragma unroll
      for (int j = 0; j < NDOF; ++j) rows[at + j] = qn[j];
    }
    // slots whose iteration this round completed: new prog, then finish
    // (write out and refill) or begin the next iteration
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (!span[s]) continue;
      pos[s] += n[s];
      if (pos[s] < cnt[s]) continue;
      its[s] += 1;
      prog[s] = uniform(prog[s] + min(first_bad[s], cnt[s]));
      const bool ok = prog[s] == W - 1;
      if (ok || its[s] >= prm.max_iters) {
        const int m = mot[s];
        __syncthreads();                 // the round's writes land before the read-out
        if (lane < W) {
#pragma unroll
          for (int j = 0; j < NDOF; ++j) xi[((int64_t)m * W + lane) * NDOF + j] = sx[s][lane][j];
        }
        if (lane == 0) {
          status[m] = ok ? 0 : 1;
          if (iters) iters[m] = (MODE == 2 ? iters[m] : 0) + (ok ? its[s] : prm.max_iters);
        }
        __syncthreads();                 // the slot is read out before it is refilled
        fetch(s);
      }
      begin_iteration(s);
    }
  }
  if (work && lane == 0) atomicAdd(&work[6], updates);
}

}  // namespace cprrtc
