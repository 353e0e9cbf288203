// Learned warm start: an MLP that predicts the projection correction dq from
// (q, constraint parameters), with BF16 weights and FP32 accumulation on the
// gfx950 matrix cores, trained on the GPU by the kernels below.
//
// Network: n_in -> hidden (SiLU) -> ... -> hidden (SiLU) -> n_out.  Every
// parameter has an FP32 master copy (Adam updates it) and a BF16 copy (the
// matrix cores read it).  Layer widths are padded inside the kernels: the
// reduction dimension to a multiple of 32 (one MFMA step), the output to a
// multiple of 16; padding is zero and never stored.
//
// Inference (and the warm start's corrections) runs the whole network in one
// launch, mlp_fused_kernel: activations never leave the registers, weights
// stream through LDS (see the comment above the kernel).
//
// Training uses one GEMM kernel for the forward pass and both backward
// products: C[M][N] = A[M][K] * B[K][N] with A and B described by strides,
// so W^T, dZ^T and X^T are read in place.  Tiles of 64 x 64 x 32 are staged in
// LDS by the whole workgroup (4 wavefronts); each wavefront computes a 32 x 32
// block as 2 x 2 v_mfma_f32_16x16x32_bf16 tiles, reading its operand
// fragments from LDS (8 consecutive BF16 per lane: A row-major, B stored
// transposed).  Epilogues fuse the bias, SiLU, and SiLU' of the backward pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <type_traits>
#include <vector>

#include "cprrtc.h"
#include "device.h"
#include "handles.h"
#include "kernels.h"
#include "project.h"

namespace cprrtc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
// SiLU with the hardware reciprocal (about 1 ulp) instead of a correctly
// rounded division; the result is rounded to BF16 right after.
__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
// SiLU'(z) = s (1 + z (1 - s)), s = sigmoid(z), with the hardware reciprocal.
__device__ __forceinline__ float silu_grad_fast(float z) {
  const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  return sg * (1.0f + z * (1.0f - sg));
}
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Operand of the GEMM: element (r, c) at p[r * rs + c * cs].
struct Mat {
  const uint16_t* p;
  long rs, cs;
};

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_SILU_GRAD = 3, EPI_PARTIAL = 4 };

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

// Loads 8 consecutive bf16 from p (16-byte aligned) as a uint4.
__device__ __forceinline__ uint4 load8(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ uint16_t lane16(const uint4& v, int i) {
  const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
  return (uint16_t)(w >> (16 * (i & 1)));
}
__device__ __forceinline__ bool aligned16(const void* p) {
  return ((uintptr_t)p & 15u) == 0;
}

// Stages the R x kBK tile of operand X (element (r, k) at p[r * rs + k * cs],
// rows r0.., reduction columns k0..) into S[r][k] (zero outside R_tot x K).
// When the reduction dimension is contiguous, a thread moves 8 consecutive
// elements of a row with one 16-byte load and store; when the row dimension
// is contiguous, 8 consecutive rows of one column with one load; otherwise
// element by element.
template <int R>
__device__ __forceinline__ void stage(uint16_t (&S)[R][kBK + kPad], const Mat& X, int r0, int k0,
                                      int R_tot, int K, int tid) {
  static_assert(R * kBK == 8 * 256, "one 8-element chunk per thread");
  if (X.cs == 1) {
    const int r = tid >> 2, c8 = (tid & 3) * 8;
    const int gr = r0 + r, gk = k0 + c8;
    const uint16_t* src = X.p + (long)gr * X.rs + gk;
    if (gr < R_tot && gk + 8 <= K && aligned16(src)) {
      *reinterpret_cast<uint4*>(&S[r][c8]) = load8(src);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        S[r][c8 + i] = (gr < R_tot && gk + i < K) ? X.p[(long)gr * X.rs + gk + i] : (uint16_t)0;
    }
  } else if (X.rs == 1) {
    const int c = tid >> 3, r8 = (tid & 7) * 8;
    const int gk = k0 + c, gr = r0 + r8;
    const uint16_t* src = X.p + gr + (long)gk * X.cs;
    if (gk < K && gr + 8 <= R_tot && aligned16(src)) {
      const uint4 v = load8(src);
#pragma unroll
      for (int i = 0; i < 8; ++i) S[r8 + i][c] = lane16(v, i);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        S[r8 + i][c] = (gk < K && gr + i < R_tot) ? X.p[(long)(gr + i) + (long)gk * X.cs] : (uint16_t)0;
    }
  } else {
    for (int e = tid; e < R * kBK; e += 256) {
      const int r = e / kBK, c = e % kBK;
      const int gr = r0 + r, gk = k0 + c;
      S[r][c] = (gr < R_tot && gk < K) ? X.p[(long)gr * X.rs + (long)gk * X.cs] : (uint16_t)0;
    }
  }
}

// C[M][N] = A[M][K] B[K][N] (+ epilogue); blockIdx.z splits the reduction
// into gridDim.z ranges of k_split (a multiple of kBK).
//  EPI_STORE:     out_f = C (fp32)
//  EPI_PARTIAL:   out_f[z][M][ldo] = this range's part of C (summed by reduce_parts_kernel)
//  EPI_BIAS:      out_f = C + bias (fp32), out_b = bf16 of it (nullable)
//  EPI_BIAS_SILU: z = C + bias -> out_f = z (pre-activation, nullable), out_b = bf16(silu(z))
//  EPI_SILU_GRAD: out_b = bf16(C * silu'(aux)) with aux the stored pre-activation
template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(Mat A, Mat B, int M, int N, int K,
                                                        int k_split,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ aux,
                                                        float* __restrict__ out_f,
                                                        uint16_t* __restrict__ out_b, long ldo) {
  __shared__ __align__(16) uint16_t As[kBM][kBK + kPad];
  __shared__ __align__(16) uint16_t Bs[kBN][kBK + kPad];   // transposed: Bs[n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;     // this wavefront's 32 x 32 block
  const int kb = blockIdx.z * k_split, ke = min(K, kb + k_split);
  // B as an operand with rows n and reduction k: element (n, k) = B(k, n)
  const Mat Bt{B.p, B.cs, B.rs};
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kb; k0 < ke; k0 += kBK) {
    stage<kBM>(As, A, m0, k0, M, ke, tid);
    stage<kBN>(Bs, Bt, n0, k0, N, ke, tid);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i)
      a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&As[wm + i * 16 + fr][fk]));
    for (int j = 0; j < 2; ++j)
      b[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bs[wn + j * 16 + fr][fk]));
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // result layout of a 16 x 16 tile: lane holds rows 4*(lane/16) + t, column lane % 16
  const int col = lane & 15, rb = (lane >> 4) * 4;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + i * 16 + rb + t, gn = n0 + wn + j * 16 + col;
        if (gm >= M || gn >= N) continue;
        const float c = acc[i][j][t];
        const long o = (long)gm * ldo + gn;
        if (EPI == EPI_STORE) {
          out_f[o] = c;
        } else if (EPI == EPI_PARTIAL) {
          out_f[(long)blockIdx.z * M * ldo + o] = c;
        } else if (EPI == EPI_BIAS) {
          const float z = c + bias[gn];
          if (out_f) out_f[o] = z;
          if (out_b) out_b[o] = to_bf16(z);
        } else if (EPI == EPI_BIAS_SILU) {
          const float z = c + bias[gn];
          if (out_f) out_f[o] = z;
          out_b[o] = to_bf16(silu(z));
        } else {
          out_b[o] = to_bf16(c * silu_grad(aux[o]));
        }
      }
}

// out[r][c] = sum over z of part[z][r][c] (c < N, row stride ld), in a fixed order.
__global__ void reduce_parts_kernel(const float* __restrict__ part, int splits, int M, int N,
                                    long ld, float* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)M * N) return;
  const long r = i / N, c = i % N, o = r * ld + c;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[(long)z * M * ld + o];
  out[o] = s;
}

// fp32 [M][n] (row stride ld_in) -> bf16 [M][ld_out], zero-padded columns n..ld_out-1
__global__ void to_bf16_kernel(const float* __restrict__ in, int M, int n, long ld_in,
                               uint16_t* __restrict__ out, int ld_out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)M * ld_out) return;
  const long m = i / ld_out;
  const int c = (int)(i % ld_out);
  out[i] = c < n ? to_bf16(in[m * ld_in + c]) : (uint16_t)0;
}

// MSE loss over the n real outputs: dy = 2 (y - t) / (M n) as bf16 [M][ld], loss sum.
__global__ void mse_grad_kernel(const float* __restrict__ y, long ldy, const float* __restrict__ t,
                                int M, int n, uint16_t* __restrict__ dy, int ld,
                                float* __restrict__ loss) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (i < (long)M * ld) {
    const long m = i / ld;
    const int c = (int)(i % ld);
    float g = 0.0f;
    if (c < n) {
      const float d = y[m * ldy + c] - t[m * n + c];
      l = d * d;
      g = 2.0f * d / ((float)M * (float)n);
    }
    dy[i] = to_bf16(g);
  }
  // wavefront sum, one atomic per wavefront
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
  if (loss && (threadIdx.x & 63) == 0) atomicAdd(loss, l / ((float)M * (float)n));
}

// bias gradient: db[n] = sum_m dz[m][n] (bf16 [M][ld]); one block per column slice
__global__ void bias_grad_kernel(const uint16_t* __restrict__ dz, int M, int N, int ld,
                                 float* __restrict__ db) {
  const int n = blockIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = threadIdx.x; m < M; m += blockDim.x) s += from_bf16(dz[(long)m * ld + n]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

// Adam on the FP32 masters, refreshing the BF16 copies.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2,
                            uint16_t* __restrict__ wb, long n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  const float upd = lr * (a / c1) / (sqrtf(v / c2) + eps);
  const float nw = w[i] - upd;
  w[i] = nw;
  wb[i] = to_bf16(nw);
}

__global__ void refresh_bf16_kernel(const float* __restrict__ w, uint16_t* __restrict__ wb, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = to_bf16(w[i]);
}

// ------------------------------------------------------------------ fused network
//
// The whole network for a tile of samples in one workgroup, activations in
// registers.  Each layer is computed transposed, H_next^T = W H^T: the
// weights are the MFMA's A operand (16 output units x 32 inputs), the
// activations its B operand (32 inputs x 16 samples), so the result tile
// leaves each lane with 4 output units (4g .. 4g+3, g = lane / 16) of one
// sample (lane % 16).  Two result tiles (units 32c .. 32c+15 and
// 32c+16 .. 32c+31) hold, in the same lane, exactly the 8 inputs that lane
// supplies to the next layer's B operand for reduction chunk c, provided the
// next layer's weights list their inputs in the matching order: B slot i of
// lane group g is input 32c + 4g + i (i < 4) or 32c + 16 + 4g + (i - 4).  The
// weights are stored once in that order (fused_weights_kernel), chunk by
// chunk in the order they are used, so no activation ever leaves the
// registers and no lane exchange is needed between layers.
//
// Workgroup: 8 wavefronts; wavefront w takes samples 16 ST w .. 16 ST (w+1)
// - 1 of the tile (ST tiles of 16 samples; ST = 512 / H from width 128 up
// keeps the register footprint the same for every width: H/2 accumulators
// and H/4 activation registers).  The weight chunks (layer rows x 32 inputs, BF16)
// stream through LDS double-buffered: the next chunk's global loads are in
// flight while the current one feeds the MFMAs, and every A fragment read
// from LDS serves ST MFMAs.  Layer 0 reads the sample features (first
// layer inputs padded to 32); the last layer has at most 16 outputs.

constexpr int kFusedWaves = 8;       // wavefronts per workgroup (4 measured 35% slower)
constexpr int kFusedMaxLayers = 9;   // at most 8 hidden layers and the output layer
// LDS position (BF16 elements) of 16-byte piece c (inputs 8c .. 8c+7) of
// row `row` of a weight chunk: rows of 64 bytes, the four pieces of a row
// permuted by bits 1-2 of the row, so that any 8 lanes of a fragment read
// (rows r .. r+7 or r+4 .. r+7 and r .. r+3 of the next piece) touch 8
// different 16-byte bank groups (measured: 0.07 M conflict cycles against
// 2.85 M with rows padded to 80 bytes).
__device__ __forceinline__ int chunk_at(int row, int c) { return row * 32 + 8 * (c ^ ((row >> 1) & 3)); }
constexpr int kFusedLdw = 32;   // LDS elements per chunk row

// The network as the fused kernel reads it.
struct FusedNet {
  const uint16_t* wf;   // weight chunks, see fused_weights_kernel
  const float* bias;    // [n_layers][H] fp32, zero past a layer's width
  int n_in, n_out, n_hidden;
};

// Position -> input index inside a 32-input chunk of a hidden-input layer.
__host__ __device__ __forceinline__ int fused_perm(int p) {
  const int g = p >> 3, i = p & 7;
  return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4);
}

// Builds the fused weight chunks from the FP32 masters.  Chunk order:
// layer 0 (H rows x 32 inputs, inputs in natural order, zero past n_in),
// then for each hidden-to-hidden layer its H/32 chunks (row-major
// [H][32]), then the last layer as one chunk (row-major [16][H], zero past
// n_out); inputs of every layer but the first in fused_perm order within
// each group of 32.
__global__ void fused_weights_kernel(const float* __restrict__ w, int H, int n_in, int n_out,
                                     int n_hidden, long w_off0, long w_off_h, long w_stride_h,
                                     long w_off_last, uint16_t* __restrict__ wf, long n_wf) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_wf) return;
  const int KC = H / 32;
  const long first = (long)H * 32;
  const long hid = (long)(n_hidden - 1) * KC * H * 32;
  float v = 0.0f;
  if (e < first) {
    const int n = (int)(e / 32), k = (int)(e % 32);
    if (k < n_in) v = w[w_off0 + (long)n * n_in + k];
  } else if (e < first + hid) {
    const long r = e - first;
    const long per_layer = (long)KC * H * 32;
    const int l = (int)(r / per_layer);
    const long rr = r % per_layer;
    const int kc = (int)(rr / ((long)H * 32));
    const int n = (int)((rr / 32) % H), p = (int)(rr % 32);
    v = w[w_off_h + l * w_stride_h + (long)n * H + kc * 32 + fused_perm(p)];
  } else {
    const long r = e - first - hid;
    const int n = (int)(r / H), c = (int)(r % H);
    if (n < n_out) v = w[w_off_last + (long)n * H + (c & ~31) + fused_perm(c & 31)];
  }
  wf[e] = to_bf16(v);
}

__global__ void fused_bias_kernel(const float* __restrict__ w, const long* __restrict__ b_off,
                                  const int* __restrict__ width, int n_layers, int H,
                                  float* __restrict__ bias) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_layers * H) return;
  const int l = i / H, n = i % H;
  bias[i] = n < width[l] ? w[b_off[l] + n] : 0.0f;
}

// Sample features from a row-major matrix x[row][ld] (n_in columns).
struct FeatRows {
  const float* x;
  long ld;
  __device__ __forceinline__ void load(long s, int k0, int n_in, float (&f)[8]) const {
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (k0 + i < n_in) ? x[s * ld + k0 + i] : 0.0f;
  }
};

// Warm-start features computed in place: row s is waypoint k = s % (W-1) + 1
// of motion s / (W-1); features = the straight-line waypoint over the joint
// range, then the constraint parameters.
struct FeatWarm {
  const float* q_from;
  const float* q_to;
  int W, dof, n_cp;
  float range[kMaxDof];
  float cp[12];
  __device__ __forceinline__ void load(long s, int k0, int n_in, float (&f)[8]) const {
    const long m = s / (W - 1);
    const int k = (int)(s % (W - 1)) + 1;
    const float t = (float)k / (float)(W - 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int c = k0 + i;
      float v = 0.0f;
      if (c < dof) {
        const float a = q_from[m * dof + c], b = q_to[m * dof + c];
        v = (a + t * (b - a)) / range[c];
      } else if (c < dof + n_cp) {
        v = cp[c - dof];
      }
      f[i] = v;
    }
  }
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// Two floats to two BF16 (round to nearest even) in one conversion.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// Registers holding one weight chunk on its way from global memory to LDS.
template <int PRE>
struct ChunkRegs {
  uint4 v[PRE];
};

// Global -> register -> LDS moves of weight chunk q in 16-byte pieces.  A
// chunk of 32 inputs: piece p = row p / 4, inputs 8 (p % 4) .. +7, LDS rows
// of kFusedLdw; the last layer (chunk q_last, 16 rows x H inputs): piece p
// = row p / (H/8), inputs 8 (p % (H/8)) .. +7, LDS rows of H + 8.
template <int H, int PRE, int NW>
struct ChunkStream {
  const uint16_t* wf;
  int q_last, tid;
  __device__ __forceinline__ int pieces(int q) const { return q < q_last ? H * 4 : 2 * H; }
  __device__ __forceinline__ int lds_at(int q, int p) const {
    return q < q_last ? chunk_at(p >> 2, p & 3) : (p / (H / 8)) * (H + 8) + (p % (H / 8)) * 8;
  }
  __device__ __forceinline__ ChunkRegs<PRE> fetch(int q) const {
    const long off = (long)q * H * 32;
    const int n = pieces(q);
    ChunkRegs<PRE> r;
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
      const int p = tid + i * NW * 64;
      r.v[i] = p < n ? *reinterpret_cast<const uint4*>(wf + off + (long)p * 8) : uint4{0, 0, 0, 0};
    }
    return r;
  }
  __device__ __forceinline__ void put(int q, const ChunkRegs<PRE>& r, uint16_t* dst) const {
    const int n = pieces(q);
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
      const int p = tid + i * NW * 64;
      if (p < n) *reinterpret_cast<uint4*>(dst + lds_at(q, p)) = r.v[i];
    }
  }
};

// What a training forward pass keeps for the backward pass and the weight
// gradients: the layer-0 inputs, every hidden layer's activation and the
// output gradient of the mean squared error, all BF16 and transposed
// (unit-major rows of ldt >= M samples, so that a 16-byte load holds 8
// consecutive samples of one unit, the matrix cores' operand layout for a
// reduction over samples); SiLU' of every hidden pre-activation (BF16, in
// the result layout of the kernels, read back by the backward pass); the
// loss (accumulated).
struct TrainIO {
  const float* target;   // [M][n_out]
  uint16_t* xt;          // [32][ldt]
  uint16_t* d;           // SiLU'(z): [block][n_hidden][wavefront][tile][lane][4]
  uint16_t* at;          // [n_hidden][H][ldt]
  uint16_t* dyt;         // [16][ldt]
  float* loss;
  float inv_mn;          // 1 / (M n_out)
  long ldt;
};

template <int H, int ST, int NW, class F>
__global__ __launch_bounds__(NW * 64) void mlp_fused_kernel(FusedNet net, F feat, long M,
                                                        float* __restrict__ y, long ldy) {
  constexpr int KC = H / 32;       // reduction chunks of a hidden-input layer
  constexpr int NT = H / 16;       // result tiles of a hidden layer
  constexpr int ROWS = H * 4;      // 16-byte pieces of a full chunk
  constexpr int PRE = (ROWS + NW * 64 - 1) / (NW * 64);
  __shared__ __align__(16) uint16_t wl[2][H * kFusedLdw];
  __shared__ __align__(16) float bias_s[kFusedMaxLayers * H];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < (net.n_hidden + 1) * H; i += NW * 64) bias_s[i] = net.bias[i];
  const int r = lane & 15, g = lane >> 4;
  const long s0 = ((long)blockIdx.x * NW + wave) * (16 * ST);
  const int q_last = 1 + (net.n_hidden - 1) * KC;   // the last layer's single chunk
  const int nq = q_last + 1;

  // Chunk q sits in LDS buffer q & 1 while it is used; chunk q + 1 is in
  // the register set (q + 1) & 1 (pre0 / pre1), loaded during the use of
  // chunk q - 1, and goes to LDS after chunk q; chunk q + 2's loads are
  // issued before chunk q is used.  Every layer but the first has an even
  // number of chunks and starts at an odd q, so the set of a chunk is known
  // at compile time.
  const ChunkStream<H, PRE, NW> cs{net.wf, q_last, tid};
  ChunkRegs<PRE> pre0 = cs.fetch(0), pre1;
  if (nq > 1) pre1 = cs.fetch(1);
  cs.put(0, pre0, wl[0]);
  __syncthreads();
  int q = 0;
  // per chunk (parity PAR = q & 1): issue chunk q + 2's loads, use chunk q,
  // store chunk q + 1, wait for every wavefront
#define FUSED_BEGIN(PAR)                                   \
  if (q + 2 < nq) {                                        \
    if (PAR == 0) pre0 = cs.fetch(q + 2);                  \
    else pre1 = cs.fetch(q + 2);                           \
  }
#define FUSED_END(PAR)                                                   \
  if (q + 1 < nq) cs.put(q + 1, PAR == 0 ? pre1 : pre0, wl[(q + 1) & 1]); \
  __syncthreads();                                                       \
  ++q;
  auto afrag = [&](int row) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&wl[q & 1][chunk_at(row, g)]));
  };

  f32x4 acc[NT][ST];
  // one chunk of a layer: every result tile takes its A fragment from LDS
  // and the B operands of this chunk's 32 inputs; the layer's first chunk
  // starts the accumulators at the bias (units 16 nt + 4g .. +3)
  auto chunk_mfma = [&](const bf16x8 (&b)[ST], int first_of_layer) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bf16x8 a = afrag(nt * 16 + r);
      if (first_of_layer >= 0) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(&bias_s[first_of_layer * H + nt * 16 + 4 * g]);
#pragma unroll
        for (int st = 0; st < ST; ++st)
          acc[nt][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[st], bv, 0, 0, 0);
      } else {
#pragma unroll
        for (int st = 0; st < ST; ++st)
          acc[nt][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[st], acc[nt][st], 0, 0, 0);
      }
    }
  };

  // layer 0: features of this lane's samples, inputs 8g .. 8g+7
  bf16x8 xin[ST];
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    const long s = s0 + st * 16 + r;
    float f[8];
    if (s < M) {
      feat.load(s, 8 * g, net.n_in, f);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) f[i] = 0.0f;
    }
    const uint4 u{pack_bf16(f[0], f[1]), pack_bf16(f[2], f[3]), pack_bf16(f[4], f[5]), pack_bf16(f[6], f[7])};
    xin[st] = __builtin_bit_cast(bf16x8, u);
  }
  FUSED_BEGIN(0)
  chunk_mfma(xin, 0);
  FUSED_END(0)

  // SiLU, then BF16 into the next layer's B operand (see above)
  bf16x8 act[KC][ST];
  auto epilogue = [&](int l) {
#pragma unroll
    for (int c = 0; c < KC; ++c) {
#pragma unroll
      for (int st = 0; st < ST; ++st) {
        const f32x4 lo = acc[2 * c][st], hi = acc[2 * c + 1][st];
        const uint4 u{pack_bf16(silu_fast(lo[0]), silu_fast(lo[1])),
                      pack_bf16(silu_fast(lo[2]), silu_fast(lo[3])),
                      pack_bf16(silu_fast(hi[0]), silu_fast(hi[1])),
                      pack_bf16(silu_fast(hi[2]), silu_fast(hi[3]))};
        act[c][st] = __builtin_bit_cast(bf16x8, u);
      }
    }
  };
  epilogue(0);

  // hidden-to-hidden layers
  for (int l = 1; l < net.n_hidden; ++l) {
    // chunks in pairs: q odd, then even
#pragma unroll
    for (int kc = 0; kc < KC; kc += 2) {
      FUSED_BEGIN(1)
      chunk_mfma(act[kc], kc == 0 ? l : -1);
      FUSED_END(1)
      FUSED_BEGIN(0)
      chunk_mfma(act[kc + 1], -1);
      FUSED_END(0)
    }
    epilogue(l);
  }

  // last layer: at most 16 outputs, bias, no activation
  const float* bl = bias_s + net.n_hidden * H;
  f32x4 out[ST];
#pragma unroll
  for (int st = 0; st < ST; ++st) out[st] = f32x4{bl[4 * g], bl[4 * g + 1], bl[4 * g + 2], bl[4 * g + 3]};
  // (the whole layer is one chunk, q = q_last: nothing left to stream)
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const bf16x8 a = __builtin_bit_cast(
        bf16x8, *reinterpret_cast<const uint4*>(&wl[q & 1][r * (H + 8) + kc * 32 + 8 * g]));
#pragma unroll
    for (int st = 0; st < ST; ++st)
      out[st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kc][st], out[st], 0, 0, 0);
  }
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    const long s = s0 + st * 16 + r;
    if (s >= M) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = 4 * g + t;
      if (n < net.n_out) y[s * ldy + n] = out[st][t];
    }
  }
#undef FUSED_BEGIN
#undef FUSED_END
}

// Training forward and backward passes for small batches.  A workgroup
// takes SB = 16 ST samples and its NW wavefronts split each layer's units
// (16 T per wavefront), so a batch of a few thousand samples still spreads
// over every CU.  A layer's input block (SB samples x its inputs, BF16) sits
// in LDS; a wavefront reads it as the A operand and its weight fragments
// straight from global memory as the B operand (the rows of its units in
// the fused chunk layout, whose input order the A reads follow), with the
// next groups of k-chunks in flight while it works on this one.  Results
// (C: unit = lane % 16, samples 4 (lane / 16) + i) go through the epilogue
// into the other LDS block, which is then written out transposed for the
// weight gradients.  SiLU' of the pre-activations is stored in the C layout
// itself (per workgroup, layer, wavefront, tile), which the backward pass
// reads with the same mapping.
// Workgroups are dispatched to the eight XCDs in turn (workgroup i to XCD
// i % 8).  The training kernels give XCD x the x-th contiguous eighth of the
// batch, so the forward pass, the backward pass and the weight-gradient
// range of the same samples run on one XCD and meet their data in its L2.
__device__ __forceinline__ long xcd_block(long i, long n) {
  return n % 8 == 0 ? (i % 8) * (n / 8) + i / 8 : i;
}

template <int H, int ST_>
struct TrainShape {
  static constexpr int NW = H >= 512 ? 16 : H >= 256 ? 8 : H / 32;   // wavefronts per workgroup
  static constexpr int T = H / (16 * NW);                    // unit tiles per wavefront
  static constexpr int KC = H / 32;                          // k-chunks of a hidden layer
  static constexpr int G = H >= 512 ? 4 : 2;                 // k-chunk groups per layer (even)
  static constexpr int GK = KC / G;                          // k-chunks per group
  static constexpr int ST = ST_;                             // 16-sample tiles per workgroup
  static constexpr int SB = 16 * ST;
  static constexpr int LDA = H + 8;                          // LDS row stride (elements)
  static constexpr int KCW = KC / NW;                        // output-layer k-chunks per wavefront
  static_assert(T >= 1 && GK >= 1 && KCW >= 1, "unsupported width");
};

// A operand: the 8 inputs of k-chunk c at fused_perm slots 8g .. 8g+7 of
// row s of an activation block (inputs 32c + 4g + 0..3 and 32c + 16 + 4g + 0..3).
template <int LDA>
__device__ __forceinline__ bf16x8 act_frag_perm(const uint16_t* blk, int s, int c, int g) {
  const uint16_t* row = blk + s * LDA + 32 * c + 4 * g;
  const uint2 lo = *reinterpret_cast<const uint2*>(row);
  const uint2 hi = *reinterpret_cast<const uint2*>(row + 16);
  return __builtin_bit_cast(bf16x8, uint4{lo.x, lo.y, hi.x, hi.y});
}
template <int LDA>
__device__ __forceinline__ bf16x8 act_frag_nat(const uint16_t* blk, int s, int g) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(blk + s * LDA + 8 * g));
}

__device__ __forceinline__ uint16_t bf16_bits(float v) { return (uint16_t)(pack_bf16(v, 0.0f) & 0xffffu); }

// Writes an LDS block (SB sample rows x W columns, row stride LDA) out
// transposed: column u to out[u * ldt + sample], 8 samples per 16-byte store.
template <int W, int SB, int LDA, int NTH>
__device__ __forceinline__ void block_out_t(const uint16_t* blk, int rows, uint16_t* out, long ldt,
                                            int tid) {
  for (int p = tid; p < W * (SB / 8); p += NTH) {
    const int u = p / (SB / 8), s8 = (p % (SB / 8)) * 8;
    uint16_t v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = blk[(s8 + i) * LDA + u];
    uint16_t* dst = out + (long)u * ldt + s8;
    if (s8 + 8 <= rows) {
      *reinterpret_cast<uint4*>(dst) =
          uint4{v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16)};
    } else {
      for (int i = 0; i < 8 && s8 + i < rows; ++i) dst[i] = v[i];
    }
  }
}

template <int H, int ST_>
__global__ __launch_bounds__((TrainShape<H, ST_>::NW * 64)) void mlp_train_fwd_kernel(FusedNet net,
                                                                             FeatRows feat, long M,
                                                                             TrainIO tr) {
  using S = TrainShape<H, ST_>;
  constexpr int NW = S::NW, T = S::T, G = S::G, GK = S::GK, ST = S::ST, SB = S::SB, LDA = S::LDA;
  constexpr int KCW = S::KCW, NTH = NW * 64;
  __shared__ __align__(16) uint16_t act[2][SB * LDA];
  __shared__ __align__(16) f32x4 red[NW][ST][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const long blk = xcd_block(blockIdx.x, gridDim.x);
  const long sb = blk * SB;
  const int rows = (int)min((long)SB, M - sb);
  const int nh = net.n_hidden;
  const int u0 = wave * 16 * T;
  const uint16_t* wh = net.wf + (long)H * 32;                          // hidden layers
  const uint16_t* wl = net.wf + (long)H * 32 + (long)(nh - 1) * H * H;  // output layer [16][H]

  // weight fragments: layer 0 and the output layer now, the first two
  // groups of the hidden layers into the two register sets
  uint4 w0[T], wo[KCW], ws0[T][GK], ws1[T][GK];
#pragma unroll
  for (int t = 0; t < T; ++t) w0[t] = *reinterpret_cast<const uint4*>(net.wf + (long)(u0 + 16 * t + r) * 32 + 8 * g);
#pragma unroll
  for (int i = 0; i < KCW; ++i)
    wo[i] = *reinterpret_cast<const uint4*>(wl + (long)r * H + 32 * (wave * KCW + i) + 8 * g);
  const int NG = (nh - 1) * G;
  auto load_group = [&](int q, uint4 (&w)[T][GK]) {
    const int l = 1 + q / G, j = q % G;
    const uint16_t* base = wh + (long)(l - 1) * H * H + (long)(j * GK) * H * 32;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int cc = 0; cc < GK; ++cc)
        w[t][cc] = *reinterpret_cast<const uint4*>(base + (long)cc * H * 32 + (long)(u0 + 16 * t + r) * 32 + 8 * g);
  };
  if (NG > 0) load_group(0, ws0);
  if (NG > 1) load_group(1, ws1);

  // layer-0 inputs: BF16 into LDS block 0 (32 columns, zero padded)
  for (int e = tid; e < SB * 32; e += NTH) {
    const int s = e / 32, k = e % 32;
    const float v = (s < rows && k < net.n_in) ? feat.x[(sb + s) * feat.ld + k] : 0.0f;
    act[0][s * LDA + k] = bf16_bits(v);
  }
  __syncthreads();
  block_out_t<32, SB, LDA, NTH>(act[0], rows, tr.xt + sb, tr.ldt, tid);

  f32x4 acc[T][ST];
  auto start = [&](int l) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float b = net.bias[l * H + u0 + 16 * t + r];
#pragma unroll
      for (int st = 0; st < ST; ++st) acc[t][st] = f32x4{b, b, b, b};
    }
  };
  // SiLU' to its store, SiLU into LDS block `out`, then the block to a_l
  auto epilogue = [&](int l, int out) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int st = 0; st < ST; ++st) {
        const f32x4 z = acc[t][st];
        const long di = ((((blk * nh + l) * NW + wave) * T + t) * ST + st) * 64 + lane;
        reinterpret_cast<uint2*>(tr.d)[di] =
            uint2{pack_bf16(silu_grad_fast(z[0]), silu_grad_fast(z[1])),
                  pack_bf16(silu_grad_fast(z[2]), silu_grad_fast(z[3]))};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          act[out][(16 * st + 4 * g + i) * LDA + u0 + 16 * t + r] = bf16_bits(silu_fast(z[i]));
      }
    __syncthreads();
    block_out_t<H, SB, LDA, NTH>(act[out], rows, tr.at + (long)l * H * tr.ldt + sb, tr.ldt, tid);
  };

  // layer 0 (one k-chunk, natural input order)
  start(0);
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    const bf16x8 a = act_frag_nat<LDA>(act[0], 16 * st + r, g);
#pragma unroll
    for (int t = 0; t < T; ++t)
      acc[t][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w0[t]), acc[t][st], 0, 0, 0);
  }
  epilogue(0, 1);
  int in = 1;
  // hidden-to-hidden layers: groups alternate between the register sets
  for (int l = 1; l < nh; ++l) {
    start(l);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int q = (l - 1) * G + j;
      auto& w = (j & 1) ? ws1 : ws0;
#pragma unroll
      for (int cc = 0; cc < GK; ++cc) {
        const int c = j * GK + cc;
#pragma unroll
        for (int st = 0; st < ST; ++st) {
          const bf16x8 a = act_frag_perm<LDA>(act[in], 16 * st + r, c, g);
#pragma unroll
          for (int t = 0; t < T; ++t)
            acc[t][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w[t][cc]), acc[t][st], 0, 0, 0);
        }
      }
      if (q + 2 < NG) load_group(q + 2, w);
    }
    epilogue(l, in ^ 1);
    in ^= 1;
  }

  // output layer: each wavefront reduces its KCW k-chunks for all 16
  // outputs, wavefront 0 sums the partials in a fixed order
  f32x4 o[ST];
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    o[st] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < KCW; ++i) {
      const bf16x8 a = act_frag_perm<LDA>(act[in], 16 * st + r, wave * KCW + i, g);
      o[st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, wo[i]), o[st], 0, 0, 0);
    }
    red[wave][st][lane] = o[st];
  }
  __syncthreads();
  if (wave != 0) return;
  // dY = 2 (y - t) / (M n_out) on the real outputs, zero on the padding:
  // output r, samples 4g .. 4g+3 of each tile (consecutive in dyt's row r)
  const float bo = r < net.n_out ? net.bias[nh * H + r] : 0.0f;
  float lsum = 0.0f;
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    f32x4 y = f32x4{bo, bo, bo, bo};
    for (int w = 0; w < NW; ++w) y += red[w][st][lane];
    float d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = 16 * st + 4 * g + i;
      d[i] = 0.0f;
      if (s < rows && r < net.n_out) d[i] = y[i] - tr.target[(sb + s) * net.n_out + r];
      lsum += d[i] * d[i];
    }
    const float k = 2.0f * tr.inv_mn;
    uint16_t* dst = tr.dyt + (long)r * tr.ldt + sb + 16 * st + 4 * g;
    if (16 * st + 4 * g + 4 <= rows) {
      *reinterpret_cast<uint2*>(dst) = uint2{pack_bf16(k * d[0], k * d[1]), pack_bf16(k * d[2], k * d[3])};
    } else {
      for (int i = 0; i < 4 && 16 * st + 4 * g + i < rows; ++i) dst[i] = bf16_bits(k * d[i]);
    }
  }
#pragma unroll
  for (int o2 = 32; o2 >= 1; o2 >>= 1) lsum += __shfl_xor(lsum, o2, 64);
  if (lane == 0) atomicAdd(tr.loss, lsum * tr.inv_mn);
}

// Backward pass for mlp_train_fwd_kernel's samples: dZ_{n_h-1} = (W_out^T
// dY) * SiLU'(z), then dZ_{l-1} = (W_l^T dZ_l) * SiLU'(z_{l-1}) down to
// layer 0, each to dzt ([n_hidden][H][ldt], BF16, transposed).  The
// transposed weights come from the backward chunks (fused_weights_t_kernel):
// the output layer's W^T ([H][32], natural order), then per hidden layer
// from the last down, H/32 chunks of [H][32] in fused_perm order.
template <int H, int ST_>
__global__ __launch_bounds__((TrainShape<H, ST_>::NW * 64)) void mlp_train_bwd_kernel(
    const uint16_t* __restrict__ wbt, int nh, long M, TrainIO tr, uint16_t* __restrict__ dzt) {
  using S = TrainShape<H, ST_>;
  constexpr int NW = S::NW, T = S::T, G = S::G, GK = S::GK, ST = S::ST, SB = S::SB, LDA = S::LDA;
  constexpr int NTH = NW * 64;
  __shared__ __align__(16) uint16_t act[2][SB * LDA];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const long blk = xcd_block(blockIdx.x, gridDim.x);
  const long sb = blk * SB;
  const int rows = (int)min((long)SB, M - sb);
  const int u0 = wave * 16 * T;
  const uint16_t* wh = wbt + (long)H * 32;
  uint4 wo[T], ws0[T][GK], ws1[T][GK];
#pragma unroll
  for (int t = 0; t < T; ++t) wo[t] = *reinterpret_cast<const uint4*>(wbt + (long)(u0 + 16 * t + r) * 32 + 8 * g);
  const int NG = (nh - 1) * G;
  // group q: product j = q / G (layer l = nh - 1 - j), k-chunks (q % G) GK ..
  auto load_group = [&](int q, uint4 (&w)[T][GK]) {
    const int j = q / G, c0 = (q % G) * GK;
    const uint16_t* base = wh + (long)j * H * H + (long)c0 * H * 32;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int cc = 0; cc < GK; ++cc)
        w[t][cc] = *reinterpret_cast<const uint4*>(base + (long)cc * H * 32 + (long)(u0 + 16 * t + r) * 32 + 8 * g);
  };
  if (NG > 0) load_group(0, ws0);
  if (NG > 1) load_group(1, ws1);

  // dY into LDS block 0 (32 columns, zero past 16)
  for (int e = tid; e < SB * 32; e += NTH) {
    const int s = e % SB, k = e / SB;
    act[0][s * LDA + k] = (s < rows && k < 16) ? tr.dyt[(long)k * tr.ldt + sb + s] : (uint16_t)0;
  }
  __syncthreads();

  f32x4 acc[T][ST];
  // dZ_l = acc * SiLU'(z_l) into LDS block `out`, then the block to dzt_l
  auto epilogue = [&](int l, int out) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int st = 0; st < ST; ++st) {
        const long di = ((((blk * nh + l) * NW + wave) * T + t) * ST + st) * 64 + lane;
        const uint2 dv = reinterpret_cast<const uint2*>(tr.d)[di];
        const float dd[4] = {__uint_as_float(dv.x << 16), __uint_as_float(dv.x & 0xffff0000u),
                             __uint_as_float(dv.y << 16), __uint_as_float(dv.y & 0xffff0000u)};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          act[out][(16 * st + 4 * g + i) * LDA + u0 + 16 * t + r] = bf16_bits(acc[t][st][i] * dd[i]);
      }
    __syncthreads();
    block_out_t<H, SB, LDA, NTH>(act[out], rows, dzt + (long)l * H * tr.ldt + sb, tr.ldt, tid);
  };

  // output layer: one k-chunk of dY (natural order)
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    const bf16x8 a = act_frag_nat<LDA>(act[0], 16 * st + r, g);
#pragma unroll
    for (int t = 0; t < T; ++t)
      acc[t][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, wo[t]),
                                                           f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
  epilogue(nh - 1, 1);
  int in = 1;
  for (int l = nh - 1; l >= 1; --l) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int st = 0; st < ST; ++st) acc[t][st] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int q = (nh - 1 - l) * G + j;
      auto& w = (j & 1) ? ws1 : ws0;
#pragma unroll
      for (int cc = 0; cc < GK; ++cc) {
        const int c = j * GK + cc;
#pragma unroll
        for (int st = 0; st < ST; ++st) {
          const bf16x8 a = act_frag_perm<LDA>(act[in], 16 * st + r, c, g);
#pragma unroll
          for (int t = 0; t < T; ++t)
            acc[t][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w[t][cc]), acc[t][st], 0, 0, 0);
        }
      }
      if (q + 2 < NG) load_group(q + 2, w);
    }
    epilogue(l - 1, in ^ 1);
    in ^= 1;
  }
}

// Builds the backward weight chunks (see mlp_train_bwd_kernel) from the
// FP32 masters.
__global__ void fused_weights_t_kernel(const float* __restrict__ w, int H, int n_out, int n_hidden,
                                       long w_off_h, long w_stride_h, long w_off_last,
                                       uint16_t* __restrict__ wbt, long n_wbt) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_wbt) return;
  const long first = (long)H * 32;
  float v = 0.0f;
  if (e < first) {
    const int k = (int)(e / 32), n = (int)(e % 32);
    if (n < n_out) v = w[w_off_last + (long)n * H + k];
  } else {
    const long r = e - first;
    const long per_layer = (long)H * H;
    const int j = (int)(r / per_layer);          // 0: the last hidden-to-hidden layer
    const long rr = r % per_layer;
    const int c = (int)(rr / ((long)H * 32));
    const int k = (int)((rr / 32) % H), p = (int)(rr % 32);
    const int l = n_hidden - 1 - j;              // hidden-to-hidden layer index 1 .. n_hidden-1
    v = w[w_off_h + (long)(l - 1) * w_stride_h + (long)(32 * c + fused_perm(p)) * H + k];
  }
  wbt[e] = to_bf16(v);
}

// The parameter index -> positions in the fused forward and backward weight
// chunks and the padded biases (-1 where a parameter has none).
struct FusedMap {
  int n_layers, H, n_in, n_out, n_hidden;
  long w_off[kFusedMaxLayers], b_off[kFusedMaxLayers];
  __device__ __forceinline__ static int inv_perm(int kk) {
    return kk < 16 ? 8 * (kk >> 2) + (kk & 3) : 8 * ((kk - 16) >> 2) + 4 + ((kk - 16) & 3);
  }
  __device__ void locate(long i, long& fwd, long& bwd, long& bias) const {
    fwd = bwd = bias = -1;
    int l = n_layers - 1;
    while (l > 0 && i < w_off[l]) --l;
    const int K = l == 0 ? n_in : H, N = l + 1 < n_layers ? H : n_out;
    if (i >= b_off[l]) {
      bias = (long)l * H + (i - b_off[l]);
      return;
    }
    const long e = i - w_off[l];
    const int n = (int)(e / K), k = (int)(e % K);
    const int KC = H / 32;
    if (l == 0) {
      fwd = (long)n * 32 + k;
    } else if (l < n_layers - 1) {
      fwd = (long)H * 32 + (long)(l - 1) * KC * H * 32 + (long)(k / 32) * H * 32 + (long)n * 32 + inv_perm(k & 31);
      bwd = (long)H * 32 + (long)(n_hidden - 1 - l) * H * H + (long)(n / 32) * H * 32 + (long)k * 32 + inv_perm(n & 31);
    } else {
      fwd = (long)H * 32 + (long)(n_hidden - 1) * H * H + (long)n * H + (k & ~31) + inv_perm(k & 31);
      bwd = (long)k * 32 + n;
    }
    (void)N;
  }
};

// What a training step updates, and how: mode 0 stores the gradient; mode
// 1 takes an Adam step on the FP32 master (learning rate lr, moments b1,
// b2, bias corrections c1, c2) and refreshes its BF16 copy, its fused
// forward and backward chunk entries and the padded bias.
struct UpdateArgs {
  int mode;
  float* grad;
  float* w;
  float* m1;
  float* m2;
  uint16_t* wb;
  uint16_t* wf;
  uint16_t* wbt;
  float* bias_f;
  FusedMap map;
  float lr, b1, b2, eps, c1, c2;
  float* loss;       // the step's loss accumulator (cleared after the hand-out)
  float* loss_out;   // nullable
};

__device__ __forceinline__ void update_param(const UpdateArgs& u, long i, float gi) {
  if (u.mode == 0) {
    u.grad[i] = gi;
    return;
  }
  const float a = u.b1 * u.m1[i] + (1.0f - u.b1) * gi;
  const float v = u.b2 * u.m2[i] + (1.0f - u.b2) * gi * gi;
  u.m1[i] = a;
  u.m2[i] = v;
  const float nw = u.w[i] - u.lr * (a / u.c1) / (sqrtf(v / u.c2) + u.eps);
  u.w[i] = nw;
  const uint16_t hb = to_bf16(nw);
  u.wb[i] = hb;
  long fwd, bwd, bias;
  u.map.locate(i, fwd, bwd, bias);
  if (fwd >= 0) u.wf[fwd] = hb;
  if (bwd >= 0) u.wbt[bwd] = hb;
  if (bias >= 0) u.bias_f[bias] = nw;
}

// Weight gradients of one training step, all layers in one launch:
// blockIdx.x = range of the batch (eight ranges: range x on XCD x, where
// the training kernels left its samples), blockIdx.y = a TM x TN tile of
// dW = dZ^T X, blockIdx.z = layer.  Each workgroup writes its range's
// partial sums into parts[range][parameter index], summed in a fixed order
// by train_update_kernel.  (Finishing a tile in the workgroup of its last
// range instead, behind a counter, needs a device-scope release per
// workgroup, which writes back the XCD's L2 each time: measured ten times
// slower than the separate launch.)
// Both operands are stored transposed (unit-major rows of ld samples), so
// every operand fragment of the matrix cores (one unit, 8 consecutive
// samples) is one 16-byte load from global memory: no LDS staging.  The
// four wavefronts of a workgroup take every fourth 32-sample step of the
// range, keep D steps of fragments in flight, and sum their partial tiles
// through LDS at the end.  The workgroups of a layer's first column of
// tiles also form its bias gradient (sums of dZ over the samples) on the
// matrix cores, as the product with a fragment of ones.
struct DwLayer {
  const uint16_t* A;   // dZ^T: (unit n, sample s) at A[n * ld + s]
  const uint16_t* B;   // X^T: (input k, sample s) at B[k * ld + s]
  int N, K;            // units, inputs
  int NA, KB;          // unit and input rows present (multiples of 16; zero past N, K)
  long w_off, b_off;
};
struct DwArgs {
  DwLayer L[kFusedMaxLayers];
  long M;         // samples
  long ld;        // row stride of the operands (>= M, a multiple of 8)
  int ks;         // samples per range (a multiple of 32)
  long n_params;
  float* parts;   // [ranges][n_params]
};

// The first lim (< 8) of the 8 BF16 values in v, zeros after.
__device__ __forceinline__ uint4 keep_first(uint4 v, int lim) {
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] &= 2 * j + 1 < lim ? 0xffffffffu : (2 * j < lim ? 0x0000ffffu : 0u);
  return uint4{w[0], w[1], w[2], w[3]};
}

template <int MI, int NI, int D>
__global__ __launch_bounds__(256) void dw_kernel(DwArgs args) {
  constexpr int TM = 16 * MI, TN = 16 * NI, NACC = MI * NI + MI;
  __shared__ f32x4 red[NACC][64];
  const DwLayer& L = args.L[blockIdx.z];
  const int tn = (L.K + TN - 1) / TN, tm = (L.N + TM - 1) / TM;
  const int tile = blockIdx.y;
  if (tile >= tm * tn) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const long kb = (long)blockIdx.x * args.ks;
  const long ke = min(kb + (long)args.ks, args.M);
  const int m0 = (tile / tn) * TM, n0 = (tile % tn) * TN;
  const bool with_bias = n0 == 0;
  const int all_steps = (int)((ke - kb + 31) / 32);
  const int ns = all_steps > wave ? (all_steps - wave + 3) / 4 : 0;   // steps wave, wave + 4, ...
  const long ld = args.ld;
  // fragment: row `row` (unit or input), samples k0 + 8g .. +7 (zero past ke)
  auto frag = [&](const uint16_t* base, int row, int avail, long k0) {
    uint4 v{0u, 0u, 0u, 0u};
    const long kk = k0 + 8 * g;
    if (row < avail && kk < ke) {
      v = *reinterpret_cast<const uint4*>(base + (long)row * ld + kk);
      if (ke - kk < 8) v = keep_first(v, (int)(ke - kk));
    }
    return v;
  };
  uint4 fa[D][MI], fb[D][NI];
  auto load = [&](int i, uint4 (&a)[MI], uint4 (&b)[NI]) {
    const long k0 = kb + 32L * (wave + 4 * i);
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) a[mi] = frag(L.A, m0 + 16 * mi + r, L.NA, k0);
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) b[ni] = frag(L.B, n0 + 16 * ni + r, L.KB, k0);
  };
  f32x4 acc[MI][NI], accb[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const uint4 one_bits{0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u};   // BF16 1.0 x 8
  const bf16x8 ones = __builtin_bit_cast(bf16x8, one_bits);
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < ns) load(d, fa[d], fb[d]);
  for (int i0 = 0; i0 < ns; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = i0 + d;
      if (i < ns) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, fa[d][mi]);
#pragma unroll
          for (int ni = 0; ni < NI; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, fb[d][ni]),
                                                                  acc[mi][ni], 0, 0, 0);
          if (with_bias) accb[mi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb[mi], 0, 0, 0);
        }
        if (i + D < ns) load(i + D, fa[d], fb[d]);
      }
    }
  }
  // wavefronts 3, 2, 1 hand their partial tiles to wavefront 0 in turn
  for (int w = 3; w >= 1; --w) {
    if (wave == w) {
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) {
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) red[mi * NI + ni][lane] = acc[mi][ni];
        red[MI * NI + mi][lane] = accb[mi];
      }
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) {
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) acc[mi][ni] += red[mi * NI + ni][lane];
        accb[mi] += red[MI * NI + mi][lane];
      }
    }
    __syncthreads();
  }
  if (wave != 0) return;
  float* out = args.parts + (long)blockIdx.x * args.n_params;
  const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + mi * 16 + rb + t, gn = n0 + ni * 16 + col;
        if (gm < L.N && gn < L.K) out[L.w_off + (long)gm * L.K + gn] = acc[mi][ni][t];
      }
    if (with_bias && col == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + mi * 16 + rb + t;
        if (gm < L.N) out[L.b_off + gm] = accb[mi][t];
      }
    }
  }
}

// Sums the ranges' partial gradients of every parameter in a fixed order
// and updates it (update_param); thread 0 also hands out the step's loss
// and clears the accumulator for the next step.
__global__ void train_update_kernel(const float* __restrict__ parts, int n_parts, long n_params,
                                    UpdateArgs u) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    if (u.loss_out) *u.loss_out = *u.loss;
    *u.loss = 0.0f;
  }
  if (i >= n_params) return;
  float gi = 0.0f;
  for (int z = 0; z < n_parts; ++z) gi += parts[(long)z * n_params + i];
  update_param(u, i, gi);
}

}  // namespace cprrtc

using namespace cprrtc;

// ------------------------------------------------------------------ the network handle

struct cp_mlp {
  int n_in = 0, hidden = 0, n_hidden = 0, n_out = 0, n_layers = 0;
  std::vector<int> in_dim, out_dim;          // per layer (unpadded)
  std::vector<long> w_off, b_off;             // offsets into the parameter vector
  long n_params = 0;
  float* w = nullptr;                         // fp32 masters [n_params]
  uint16_t* wb = nullptr;                     // bf16 copies
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  long step = 0;
  // activation workspace for up to ws_rows rows
  long ws_rows = 0;
  uint16_t* xb = nullptr;                     // [rows][in_pad]
  std::vector<uint16_t*> hb;                  // per layer output, bf16 [rows][out_pad]
  std::vector<float*> zf;                     // per hidden layer pre-activation fp32 [rows][hidden]
  float* yf = nullptr;                        // [rows][out_pad] fp32
  uint16_t* dyb = nullptr;                    // [rows][max_pad] bf16 gradient buffers
  uint16_t* dzb = nullptr;
  float* loss = nullptr;
  // inference workspace (chunked, no stored pre-activations)
  long inf_rows = 0;
  uint16_t* ia = nullptr;                     // [rows][max width] bf16, ping
  uint16_t* ib = nullptr;                     // pong
  uint16_t* ix = nullptr;                     // [rows][in_pad] bf16 input
  float* iy = nullptr;                        // [rows][out_pad] fp32 output
  float* parts = nullptr;                     // split-reduction parts of the weight gradients
  long parts_cap = 0;                         // floats
  float* feat = nullptr;                      // warm start: [rows][n_in] features
  float* delta = nullptr;                     // warm start: [rows][n_out] corrections
  long warm_rows = 0;
  // fused network (mlp_fused_kernel): BF16 weight chunks and padded biases,
  // rebuilt from the masters whenever they change
  bool fusable = false;
  uint16_t* wf = nullptr;
  long n_wf = 0;
  float* bias_f = nullptr;
  long* d_b_off = nullptr;
  int* d_width = nullptr;
  // fused training: backward weight chunks and the step's buffers
  uint16_t* wbt = nullptr;
  long n_wbt = 0;
  long tr_rows = 0;
  uint16_t* t_xt = nullptr;   // [32][rows]
  uint16_t* t_d = nullptr;    // SiLU' of the pre-activations, [n_hidden][rows][H]
  uint16_t* t_at = nullptr;   // [n_hidden][H][rows]
  uint16_t* t_dyt = nullptr;  // [16][rows]
  uint16_t* t_dzt = nullptr;  // [n_hidden][H][rows]
  float* t_parts = nullptr;   // [kTrainParts][n_params]
};

namespace {

int pad32(int x) { return (x + 31) / 32 * 32; }
int pad16(int x) { return (x + 15) / 16 * 16; }

void free_ws(cp_mlp* n) {
  if (n->xb) (void)hipFree(n->xb);
  for (auto p : n->hb) if (p) (void)hipFree(p);
  for (auto p : n->zf) if (p) (void)hipFree(p);
  if (n->yf) (void)hipFree(n->yf);
  if (n->dyb) (void)hipFree(n->dyb);
  if (n->dzb) (void)hipFree(n->dzb);
  n->xb = nullptr;
  n->hb.assign(n->hb.size(), nullptr);
  n->zf.assign(n->zf.size(), nullptr);
  n->yf = nullptr;
  n->dyb = n->dzb = nullptr;
  n->ws_rows = 0;
}

// width used for a layer's output buffer: hidden layers keep their width
// (a multiple of 32), the last layer is padded to 16 columns
int out_pad(const cp_mlp* n, int l) { return l + 1 < n->n_layers ? n->out_dim[l] : pad16(n->out_dim[l]); }
int in_pad(const cp_mlp* n) { return pad32(n->n_in); }

hipError_t ensure_ws(cp_mlp* n, long rows) {
  if (rows <= n->ws_rows) return hipSuccess;
  free_ws(n);
  long r = std::max(rows, 256L);
  hipError_t e = hipMalloc((void**)&n->xb, sizeof(uint16_t) * r * in_pad(n));
  n->hb.assign(n->n_layers, nullptr);
  n->zf.assign(n->n_layers, nullptr);
  int maxw = in_pad(n);
  for (int l = 0; l < n->n_layers && e == hipSuccess; ++l) {
    e = hipMalloc((void**)&n->hb[l], sizeof(uint16_t) * r * out_pad(n, l));
    if (e == hipSuccess && l + 1 < n->n_layers) e = hipMalloc((void**)&n->zf[l], sizeof(float) * r * n->out_dim[l]);
    maxw = std::max(maxw, out_pad(n, l));
  }
  if (e == hipSuccess) e = hipMalloc((void**)&n->yf, sizeof(float) * r * out_pad(n, n->n_layers - 1));
  if (e == hipSuccess) e = hipMalloc((void**)&n->dyb, sizeof(uint16_t) * r * maxw);
  if (e == hipSuccess) e = hipMalloc((void**)&n->dzb, sizeof(uint16_t) * r * maxw);
  if (e == hipSuccess && !n->parts) {
    long wmax = 0;
    for (int l = 0; l < n->n_layers; ++l) wmax = std::max(wmax, (long)n->out_dim[l] * n->in_dim[l]);
    n->parts_cap = 32 * wmax;
    e = hipMalloc((void**)&n->parts, sizeof(float) * n->parts_cap);
  }
  if (e == hipSuccess) n->ws_rows = r;
  return e;
}

void gemm(int epi, Mat A, Mat B, int M, int N, int K, const float* bias, const float* aux,
          float* out_f, uint16_t* out_b, long ldo, hipStream_t st) {
  dim3 grid((M + kBM - 1) / kBM, (N + kBN - 1) / kBN, 1);
  const int ks = (K + kBK - 1) / kBK * kBK;
  switch (epi) {
    case EPI_STORE: gemm_bf16_kernel<EPI_STORE><<<grid, 256, 0, st>>>(A, B, M, N, K, ks, bias, aux, out_f, out_b, ldo); break;
    case EPI_BIAS: gemm_bf16_kernel<EPI_BIAS><<<grid, 256, 0, st>>>(A, B, M, N, K, ks, bias, aux, out_f, out_b, ldo); break;
    case EPI_BIAS_SILU: gemm_bf16_kernel<EPI_BIAS_SILU><<<grid, 256, 0, st>>>(A, B, M, N, K, ks, bias, aux, out_f, out_b, ldo); break;
    default: gemm_bf16_kernel<EPI_SILU_GRAD><<<grid, 256, 0, st>>>(A, B, M, N, K, ks, bias, aux, out_f, out_b, ldo); break;
  }
}

unsigned nblk(long n, int b = 256);

// C = A B stored to out_f (fp32, row stride ldo) with the reduction split
// over enough workgroups to fill the chip when the output is small and the
// reduction long (the weight gradients: output = layer size, reduction =
// batch); parts go to `parts` ([splits][M][ldo] fp32) and are summed in a
// fixed order, so the result does not depend on scheduling.
void gemm_split(Mat A, Mat B, int M, int N, int K, float* out_f, long ldo, float* parts,
                long parts_cap, hipStream_t st) {
  const int tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  const int ksteps = (K + kBK - 1) / kBK;
  int splits = std::min(std::max(1, 1024 / tiles), std::max(1, ksteps / 4));
  while (splits > 1 && (long)splits * M * ldo > parts_cap) --splits;
  if (splits == 1) {
    gemm(EPI_STORE, A, B, M, N, K, nullptr, nullptr, out_f, nullptr, ldo, st);
    return;
  }
  const int ks = (ksteps + splits - 1) / splits * kBK;
  splits = (K + ks - 1) / ks;
  dim3 grid((M + kBM - 1) / kBM, (N + kBN - 1) / kBN, splits);
  gemm_bf16_kernel<EPI_PARTIAL><<<grid, 256, 0, st>>>(A, B, M, N, K, ks, nullptr, nullptr, parts, nullptr, ldo);
  reduce_parts_kernel<<<nblk((long)M * N), 256, 0, st>>>(parts, splits, M, N, ldo, out_f);
}

unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// Forward of M rows; x: fp32 [M][n_in] (row stride ldx).  Leaves activations
// in the workspace; the network output (fp32) is n->yf [M][out_pad].
hipError_t forward(cp_mlp* n, long M, const float* x, long ldx, hipStream_t st) {
  hipError_t e = ensure_ws(n, M);
  if (e != hipSuccess) return e;
  const int ip = in_pad(n);
  to_bf16_kernel<<<nblk(M * ip), 256, 0, st>>>(x, (int)M, n->n_in, ldx, n->xb, ip);
  const uint16_t* in = n->xb;
  long ld_in = ip;
  for (int l = 0; l < n->n_layers; ++l) {
    const int K = n->in_dim[l], N = n->out_dim[l];
    Mat A{in, ld_in, 1};
    Mat B{n->wb + n->w_off[l], 1, (long)K};       // B[k][n] = W[n][k]
    const float* bias = n->w + n->b_off[l];
    if (l + 1 < n->n_layers) {
      gemm(EPI_BIAS_SILU, A, B, (int)M, N, K, bias, nullptr, n->zf[l], n->hb[l], out_pad(n, l), st);
    } else {
      gemm(EPI_BIAS, A, B, (int)M, N, K, bias, nullptr, n->yf, nullptr, out_pad(n, l), st);
    }
    in = n->hb[l];
    ld_in = out_pad(n, l);
  }
  return hipGetLastError();
}

// Backward of the MSE loss after forward(): gradients into n->grad.
hipError_t backward(cp_mlp* n, long M, const float* t, hipStream_t st) {
  const int L = n->n_layers;
  const int op = out_pad(n, L - 1);
  if (n->loss) (void)hipMemsetAsync(n->loss, 0, sizeof(float), st);
  mse_grad_kernel<<<nblk(M * op), 256, 0, st>>>(n->yf, op, t, (int)M, n->n_out, n->dyb, op, n->loss);
  uint16_t* dz = n->dyb;      // gradient wrt the current layer's output pre-activation
  int ldz = op;
  for (int l = L - 1; l >= 0; --l) {
    const int K = n->in_dim[l], N = n->out_dim[l];
    const uint16_t* in = l == 0 ? n->xb : n->hb[l - 1];
    const long ld_in = l == 0 ? in_pad(n) : out_pad(n, l - 1);
    // dW[N][K] = dZ^T[N][M] * X[M][K], the batch reduction split over workgroups
    gemm_split(Mat{dz, 1, (long)ldz}, Mat{in, ld_in, 1}, N, K, (int)M, n->grad + n->w_off[l], K,
               n->parts, n->parts_cap, st);
    bias_grad_kernel<<<N, 256, 0, st>>>(dz, (int)M, N, ldz, n->grad + n->b_off[l]);
    if (l == 0) break;
    // dH[M][K] = dZ[M][N] * W[N][K], then dZ_prev = dH * silu'(z_prev)
    uint16_t* next = (dz == n->dyb) ? n->dzb : n->dyb;
    gemm(EPI_SILU_GRAD, Mat{dz, (long)ldz, 1}, Mat{n->wb + n->w_off[l], (long)K, 1}, (int)M, K, N,
         nullptr, n->zf[l - 1], nullptr, next, K, st);
    dz = next;
    ldz = K;
  }
  return hipGetLastError();
}

// The fused kernel covers hidden widths 64 .. 512 (powers of two), at most
// 32 inputs and 16 outputs.
bool fusable(int n_in, int hidden, int n_out) {
  return n_in <= 32 && n_out <= 16 && (hidden == 64 || hidden == 128 || hidden == 256 || hidden == 512);
}

long fused_weight_count(const cp_mlp* n) {
  const int H = n->hidden;
  return (long)H * 32 + (long)(n->n_hidden - 1) * H * H + (long)H / 32 * 16 * 32;
}

// Rebuilds the fused weight chunks and biases from the FP32 masters.
hipError_t refresh_fused(cp_mlp* n, hipStream_t st) {
  if (!n->fusable) return hipSuccess;
  const long w_off_h = n->n_hidden > 1 ? n->w_off[1] : 0;
  const long w_stride_h = n->n_hidden > 2 ? n->w_off[2] - n->w_off[1] : 0;
  fused_weights_kernel<<<nblk(n->n_wf), 256, 0, st>>>(n->w, n->hidden, n->n_in, n->n_out, n->n_hidden,
                                                      n->w_off[0], w_off_h, w_stride_h,
                                                      n->w_off[n->n_hidden], n->wf, n->n_wf);
  fused_bias_kernel<<<nblk((long)n->n_layers * n->hidden), 256, 0, st>>>(
      n->w, n->d_b_off, n->d_width, n->n_layers, n->hidden, n->bias_f);
  fused_weights_t_kernel<<<nblk(n->n_wbt), 256, 0, st>>>(n->w, n->hidden, n->n_out, n->n_hidden,
                                                        w_off_h, w_stride_h, n->w_off[n->n_hidden],
                                                        n->wbt, n->n_wbt);
  return hipGetLastError();
}

constexpr int kTrainParts = 8;    // batch ranges of the weight-gradient launch (one per XCD)


// Row stride of the transposed training buffers: M rounded up to 32 (the
// weight-gradient steps, which also covers the workgroups' 16-sample
// blocks), plus 64 samples so that consecutive rows start 128 bytes apart
// modulo a power of two and spread over the memory channels.
long train_ld(long M) { return (M + 31) / 32 * 32 + 64; }

void free_train(cp_mlp* n) {
  for (void* p : {(void*)n->t_xt, (void*)n->t_d, (void*)n->t_at, (void*)n->t_dyt, (void*)n->t_dzt})
    if (p) (void)hipFree(p);
  n->t_xt = n->t_d = n->t_at = n->t_dyt = n->t_dzt = nullptr;
  n->tr_rows = 0;
}

hipError_t ensure_train(cp_mlp* n, long M) {
  hipError_t e = hipSuccess;
  if (!n->t_parts) e = hipMalloc((void**)&n->t_parts, sizeof(float) * kTrainParts * n->n_params);

  if (e != hipSuccess || train_ld(M) <= n->tr_rows) return e;
  free_train(n);
  const long r = train_ld(std::max(M, 256L)), H = n->hidden, L = n->n_hidden;
  e = hipMalloc((void**)&n->t_xt, sizeof(uint16_t) * r * 32);
  if (e == hipSuccess) e = hipMalloc((void**)&n->t_d, sizeof(uint16_t) * L * r * H);
  if (e == hipSuccess) e = hipMalloc((void**)&n->t_at, sizeof(uint16_t) * L * r * H);
  if (e == hipSuccess) e = hipMalloc((void**)&n->t_dyt, sizeof(uint16_t) * r * 16);
  if (e == hipSuccess) e = hipMalloc((void**)&n->t_dzt, sizeof(uint16_t) * L * r * H);
  if (e == hipSuccess) n->tr_rows = r;
  return e;
}

template <int H, int ST>
void launch_train_hs(const cp_mlp* n, long M, const float* x, const TrainIO& tr, hipStream_t st) {
  using S = TrainShape<H, ST>;
  const unsigned blocks = (unsigned)((M + S::SB - 1) / S::SB);
  FusedNet net{n->wf, n->bias_f, n->n_in, n->n_out, n->n_hidden};
  mlp_train_fwd_kernel<H, ST><<<blocks, S::NW * 64, 0, st>>>(net, FeatRows{x, n->n_in}, M, tr);
  mlp_train_bwd_kernel<H, ST><<<blocks, S::NW * 64, 0, st>>>(n->wbt, n->n_hidden, M, tr, n->t_dzt);
}

// 16 samples per workgroup up to 8192 (every CU busy; measured faster at
// 4096), 32 above (half the weight traffic; measured 13-22% faster at 16384)
template <int H>
void launch_train_h(const cp_mlp* n, long M, const float* x, const TrainIO& tr, hipStream_t st) {
  if (M <= 8192) launch_train_hs<H, 1>(n, M, x, tr, st);
  else launch_train_hs<H, 2>(n, M, x, tr, st);
}

// One training step (mode 1: Adam with learning rate lr and bias corrections
// c1, c2) or the gradients alone (mode 0, into d_grad) of the mean squared
// error over M samples, in four launches: forward (keeping what the backward
// pass needs), backward, the weight gradients of every layer, the update.
hipError_t fused_train(cp_mlp* n, long M, const float* x, const float* t, int mode, float* d_grad,
                       float* d_loss, float lr, float c1, float c2, hipStream_t st) {
  hipError_t e = ensure_train(n, M);
  if (e != hipSuccess) return e;
  const int H = n->hidden, L = n->n_hidden;
  const long ldt = train_ld(M);
  TrainIO tr{t, n->t_xt, n->t_d, n->t_at, n->t_dyt, n->loss, 1.0f / ((float)M * (float)n->n_out), ldt};
  switch (H) {
    case 64: launch_train_h<64>(n, M, x, tr, st); break;
    case 128: launch_train_h<128>(n, M, x, tr, st); break;
    case 256: launch_train_h<256>(n, M, x, tr, st); break;
    default: launch_train_h<512>(n, M, x, tr, st); break;
  }
  // weight and bias gradients of every layer, in batch ranges
  DwArgs da;
  std::memset(&da, 0, sizeof da);
  // eight batch ranges, one per XCD
  const int ks = (int)(((M + 7) / 8 + kBK - 1) / kBK * kBK);
  const int parts = (int)((M + ks - 1) / ks);
  da.M = M;
  da.ld = ldt;
  da.ks = ks;
  da.n_params = n->n_params;
  da.parts = n->t_parts;
  // 32 x 32 tiles (more workgroups, two steps in flight; measured against
  // four steps, 64 x 64 and 32 x 64 tiles and 4 or 16 ranges) for batches of
  // a few thousand samples, 64 x 64 above
  const bool small = M <= 8192;
  const int MI = small ? 2 : 4, NI = MI, TM = 16 * MI, TN = 16 * NI;
  int max_tiles = 0;
  for (int l = 0; l < n->n_layers; ++l) {
    DwLayer& D = da.L[l];
    const bool last = l + 1 == n->n_layers;
    D.N = n->out_dim[l];
    D.K = n->in_dim[l];
    D.NA = last ? 16 : H;
    D.KB = l == 0 ? 32 : H;
    D.w_off = n->w_off[l];
    D.b_off = n->b_off[l];
    D.A = last ? n->t_dyt : n->t_dzt + (long)l * H * ldt;
    D.B = l == 0 ? n->t_xt : n->t_at + (long)(l - 1) * H * ldt;
    max_tiles = std::max(max_tiles, ((D.N + TM - 1) / TM) * ((D.K + TN - 1) / TN));
  }
  UpdateArgs u;
  std::memset(&u, 0, sizeof u);
  u.mode = mode;
  u.grad = d_grad;
  u.w = n->w;
  u.m1 = n->m1;
  u.m2 = n->m2;
  u.wb = n->wb;
  u.wf = n->wf;
  u.wbt = n->wbt;
  u.bias_f = n->bias_f;
  u.map.n_layers = n->n_layers;
  u.map.H = H;
  u.map.n_in = n->n_in;
  u.map.n_out = n->n_out;
  u.map.n_hidden = L;
  for (int l = 0; l < n->n_layers; ++l) {
    u.map.w_off[l] = n->w_off[l];
    u.map.b_off[l] = n->b_off[l];
  }
  u.lr = lr;
  u.b1 = 0.9f;
  u.b2 = 0.999f;
  u.eps = 1e-8f;
  u.c1 = c1;
  u.c2 = c2;
  u.loss = n->loss;
  u.loss_out = d_loss;
  const dim3 grid(parts, max_tiles, n->n_layers);
  if (small) dw_kernel<2, 2, 2><<<grid, 256, 0, st>>>(da);
  else dw_kernel<4, 4, 2><<<grid, 256, 0, st>>>(da);
  train_update_kernel<<<nblk(n->n_params), 256, 0, st>>>(n->t_parts, parts, n->n_params, u);
  return hipGetLastError();
}

template <int H, class F>
void launch_fused_h(const cp_mlp* n, const F& feat, long M, float* y, long ldy, hipStream_t st) {
  constexpr int ST = H >= 128 ? 512 / H : 4;
  constexpr int NW = kFusedWaves;
  const long per = (long)NW * 16 * ST;
  const unsigned blocks = (unsigned)((M + per - 1) / per);
  FusedNet net{n->wf, n->bias_f, n->n_in, n->n_out, n->n_hidden};
  mlp_fused_kernel<H, ST, NW, F><<<blocks, NW * 64, 0, st>>>(net, feat, M, y, ldy);
}

// y[M][ldy] (first n_out columns) = network(features) in one launch.
template <class F>
hipError_t infer_fused(const cp_mlp* n, const F& feat, long M, float* y, long ldy, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  switch (n->hidden) {
    case 64: launch_fused_h<64>(n, feat, M, y, ldy, st); break;
    case 128: launch_fused_h<128>(n, feat, M, y, ldy, st); break;
    case 256: launch_fused_h<256>(n, feat, M, y, ldy, st); break;
    default: launch_fused_h<512>(n, feat, M, y, ldy, st); break;
  }
  return hipGetLastError();
}

constexpr long kInferChunk = 1L << 19;   // rows per inference chunk

hipError_t ensure_infer(cp_mlp* n) {
  if (n->inf_rows) return hipSuccess;
  const long r = kInferChunk;
  int maxw = 0;
  for (int l = 0; l < n->n_layers; ++l) maxw = std::max(maxw, out_pad(n, l));
  hipError_t e = hipMalloc((void**)&n->ia, sizeof(uint16_t) * r * maxw);
  if (e == hipSuccess) e = hipMalloc((void**)&n->ib, sizeof(uint16_t) * r * maxw);
  if (e == hipSuccess) e = hipMalloc((void**)&n->ix, sizeof(uint16_t) * r * in_pad(n));
  if (e == hipSuccess) e = hipMalloc((void**)&n->iy, sizeof(float) * r * out_pad(n, n->n_layers - 1));
  if (e == hipSuccess) n->inf_rows = r;
  return e;
}

// y[M][n_out] = network(x[M][n_in]): one fused launch when the shape allows,
// else layer by layer in chunks of kInferChunk rows.
hipError_t infer(cp_mlp* n, long M, const float* x, float* y, hipStream_t st) {
  if (n->fusable) return infer_fused(n, FeatRows{x, n->n_in}, M, y, n->n_out, st);
  hipError_t e = ensure_infer(n);
  const int ip = in_pad(n), op = out_pad(n, n->n_layers - 1);
  for (long r0 = 0; r0 < M && e == hipSuccess; r0 += kInferChunk) {
    const long R = std::min(kInferChunk, M - r0);
    to_bf16_kernel<<<nblk(R * ip), 256, 0, st>>>(x + r0 * n->n_in, (int)R, n->n_in, n->n_in, n->ix, ip);
    const uint16_t* in = n->ix;
    long ld_in = ip;
    uint16_t* bufs[2] = {n->ia, n->ib};
    for (int l = 0; l < n->n_layers; ++l) {
      const int K = n->in_dim[l], N = n->out_dim[l];
      Mat A{in, ld_in, 1};
      Mat B{n->wb + n->w_off[l], 1, (long)K};
      const float* bias = n->w + n->b_off[l];
      if (l + 1 < n->n_layers) {
        gemm(EPI_BIAS_SILU, A, B, (int)R, N, K, bias, nullptr, nullptr, bufs[l & 1], out_pad(n, l), st);
        in = bufs[l & 1];
        ld_in = out_pad(n, l);
      } else {
        gemm(EPI_BIAS, A, B, (int)R, N, K, bias, nullptr, n->iy, nullptr, op, st);
      }
    }
    e = hipMemcpy2DAsync(y + r0 * n->n_out, sizeof(float) * n->n_out, n->iy, sizeof(float) * op,
                         sizeof(float) * n->n_out, R, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

}  // namespace

// Features of the warm start, one row per waypoint k = 1..W-1 of each
// motion: the straight-line waypoint scaled by the joint range, then the
// constraint parameters (pose: locked targets; relative pose: p* and R*).
template <int NDOF>
__global__ void warm_features_kernel(const RobotDev* __restrict__ rob, int W, int n_motions,
                                     const float* __restrict__ q_from,
                                     const float* __restrict__ q_to, const float* __restrict__ cp,
                                     int n_cp, float* __restrict__ x) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (long)n_motions * (W - 1)) return;
  const long m = row / (W - 1);
  const int k = (int)(row % (W - 1)) + 1;
  const float s = (float)k / (float)(W - 1);
  float* o = x + row * (NDOF + n_cp);
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    const float a = q_from[m * NDOF + j], b = q_to[m * NDOF + j];
    const float range = fmaxf(fabsf(rob->lo[j]), fabsf(rob->hi[j]));
    o[j] = (a + s * (b - a)) / range;
  }
  for (int c = 0; c < n_cp; ++c) o[NDOF + c] = cp[c];
}

// Training pairs of the warm start from projected motions: row
// m (W-1) + k - 1 holds the features of waypoint k of motion m (as the
// warm start computes them) and its target, the projected waypoint minus the
// straight-line one.
template <int NDOF>
__global__ void warm_pairs_kernel(FeatWarm f, long rows, const float* __restrict__ xi,
                                  float* __restrict__ x, float* __restrict__ t) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const int n_in = NDOF + f.n_cp;
  for (int k0 = 0; k0 < n_in; k0 += 8) {
    float v[8];
    f.load(row, k0, n_in, v);
    for (int i = 0; i < 8 && k0 + i < n_in; ++i) x[row * n_in + k0 + i] = v[i];
  }
  const long m = row / (f.W - 1);
  const int k = (int)(row % (f.W - 1)) + 1;
  const float s = (float)k / (float)(f.W - 1);
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    const float a = f.q_from[m * NDOF + j], b = f.q_to[m * NDOF + j];
    t[row * NDOF + j] = xi[(m * f.W + k) * NDOF + j] - (a + s * (b - a));
  }
}

namespace cprrtc {
// feature count of the warm start for a robot and constraint
int warm_inputs(int dof, int kind) { return dof + (kind == KIND_REL ? 12 : 6); }
}  // namespace cprrtc

namespace {

// Constraint parameters given to the network (pose: the locked targets;
// relative pose: p* and R* row-major); returns their count.
int warm_params(const ConDev& con, float (&cp)[12]) {
  for (float& v : cp) v = 0.0f;
  if (con.kind == KIND_REL) {
    for (int i = 0; i < 3; ++i) cp[i] = con.target[i];
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) cp[3 + 3 * i + c] = con.Rt[3 * c + i];   // R* row-major
    return 12;
  }
  if (con.kind == KIND_POSE)
    for (int i = 0; i < 6; ++i) cp[i] = con.target[i] * con.mask[i];
  return 6;
}

FeatWarm warm_feat(const cp_robot* robot, const ConDev& con, int W, const float* q_from,
                   const float* q_to) {
  FeatWarm f;
  f.q_from = q_from;
  f.q_to = q_to;
  f.W = W;
  f.dof = robot->host.dof;
  for (int j = 0; j < kMaxDof; ++j) {
    f.range[j] = j < f.dof ? std::fmax(std::fabs(robot->host.lo[j]), std::fabs(robot->host.hi[j])) : 1.0f;
  }
  f.n_cp = warm_params(con, f.cp);
  return f;
}

// The projection from the corrected waypoints (network output delta
// [motion][W-1][dof]), then, unless CP_WARM_NO_FALLBACK, the plain projector
// on every motion the warm pass did not project.
int warm_project(const cp_robot* robot, const ConDev& con, const cp_proj_params& p,
                 const float* delta, int32_t n_motions, const float* d_q_from, const float* d_q_to,
                 float* d_xi, int32_t* d_status, int32_t* d_iters, uint64_t* d_work, int32_t flags,
                 hipStream_t st) {
  ProjDev prm;
  prm.W = p.W;
  prm.max_iters = p.max_iters;
  prm.tau = (float)p.tau;
  prm.tau_sm = (float)p.tau_sm;
  prm.tau_task = (float)p.tau_task;
  prm.alpha = (float)p.alpha;
  prm.lambda2 = (float)(p.lambda * p.lambda);
  prm.variant = p.variant;
  const int dof = robot->host.dof;
  bool sup = false;
  hipError_t e = launch_project_mode(dof, 1, robot->dev, con, prm, n_motions, d_q_from, d_q_to, delta,
                                     d_xi, d_status, d_iters, (unsigned long long*)d_work, -1, st, &sup);
  if (e == hipSuccess && sup && !(flags & CP_WARM_NO_FALLBACK))
    e = launch_project_mode(dof, 2, robot->dev, con, prm, n_motions, d_q_from, d_q_to, nullptr,
                            d_xi, d_status, d_iters, (unsigned long long*)d_work, -1, st, &sup);
  if (!sup) return api_fail(CP_E_UNSUPPORTED, "no kernel for dof %d with constraint kind %d", dof, con.kind);
  if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm projection");
  return CP_OK;
}

// Device memory of project_motions_warm_noalloc: the network's corrections
// [rows][dof] live in this fixed array (one copy per GPU, held until the
// process ends) instead of memory the library allocates.
constexpr long kNoAllocFloats = 8L << 20;   // 32 MiB
static __device__ __align__(256) float scratch[kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex scratch_lock;
float* scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (the array's name is a host-side stand-in, not a device address).
hipError_t scratch_address(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_lock);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace cprrtc {

int mlp_warm_check(const cp_mlp* mlp, int dof, int kind) {
  if (mlp->n_in != warm_inputs(dof, kind) || mlp->n_out != dof)
    return api_fail(CP_E_ARG, "network has %d inputs / %d outputs, the warm start needs %d / %d",
                    mlp->n_in, mlp->n_out, warm_inputs(dof, kind), dof);
  if (!mlp->fusable)
    return api_fail(CP_E_UNSUPPORTED, "the planners' warm start needs a fused network shape "
                    "(hidden 64/128/256/512, at most 32 inputs and 16 outputs)");
  return CP_OK;
}

hipError_t mlp_warm_corrections(const cp_mlp* mlp, const cp_robot* robot, const ConDev& con, int W,
                                long n_segments, const float* q_from, const float* q_to,
                                float* delta, hipStream_t st) {
  return infer_fused(mlp, warm_feat(robot, con, W, q_from, q_to), n_segments * (W - 1), delta,
                     robot->host.dof, st);
}

}  // namespace cprrtc

extern "C" {

int cp_mlp_create(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out, uint64_t seed,
                  cp_mlp** out) {
  try {
    if (!out) return api_fail(CP_E_ARG, "cp_mlp_create: NULL argument");
    *out = nullptr;
    if (n_in < 1 || n_in > 256 || n_out < 1 || n_out > 256 || n_hidden < 1 || n_hidden > 8 ||
        hidden < 32 || hidden > 2048 || hidden % 32)
      return api_fail(CP_E_ARG, "cp_mlp_create: sizes out of range (hidden a multiple of 32)");
    cp_mlp* n = new (std::nothrow) cp_mlp;
    if (!n) return api_fail(CP_E_ARG, "out of host memory");
    n->n_in = n_in; n->hidden = hidden; n->n_hidden = n_hidden; n->n_out = n_out;
    n->n_layers = n_hidden + 1;
    long off = 0;
    for (int l = 0; l < n->n_layers; ++l) {
      const int K = l == 0 ? n_in : hidden, N = l + 1 < n->n_layers ? hidden : n_out;
      n->in_dim.push_back(K);
      n->out_dim.push_back(N);
      n->w_off.push_back(off);
      off += (long)N * K;
      n->b_off.push_back(off);
      off += N;
    }
    n->n_params = off;
    // He-style uniform initialisation from the seed, zero biases
    std::vector<float> w(off, 0.0f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < n->n_layers; ++l) {
      const float a = std::sqrt(6.0f / (float)n->in_dim[l]) * (l + 1 < n->n_layers ? 1.0f : 0.1f);
      std::uniform_real_distribution<float> u(-a, a);
      for (long i = 0; i < (long)n->in_dim[l] * n->out_dim[l]; ++i) w[n->w_off[l] + i] = u(rng);
    }
    hipError_t e = hipMalloc((void**)&n->w, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc((void**)&n->wb, sizeof(uint16_t) * off);
    if (e == hipSuccess) e = hipMalloc((void**)&n->grad, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc((void**)&n->m1, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc((void**)&n->m2, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc((void**)&n->loss, sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(n->w, w.data(), sizeof(float) * off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->loss, 0, sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->m1, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(n->m2, 0, sizeof(float) * off);
    n->fusable = fusable(n_in, hidden, n_out);
    if (e == hipSuccess && n->fusable) {
      n->n_wf = fused_weight_count(n);
      n->n_wbt = (long)hidden * 32 + (long)(n_hidden - 1) * hidden * hidden;
      std::vector<int> width(n->out_dim);
      e = hipMalloc((void**)&n->wf, sizeof(uint16_t) * n->n_wf);
      if (e == hipSuccess) e = hipMalloc((void**)&n->wbt, sizeof(uint16_t) * n->n_wbt);
      if (e == hipSuccess) e = hipMalloc((void**)&n->bias_f, sizeof(float) * n->n_layers * hidden);
      if (e == hipSuccess) e = hipMalloc((void**)&n->d_b_off, sizeof(long) * n->n_layers);
      if (e == hipSuccess) e = hipMalloc((void**)&n->d_width, sizeof(int) * n->n_layers);
      if (e == hipSuccess)
        e = hipMemcpy(n->d_b_off, n->b_off.data(), sizeof(long) * n->n_layers, hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(n->d_width, width.data(), sizeof(int) * n->n_layers, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
      refresh_bf16_kernel<<<nblk(off), 256>>>(n->w, n->wb, off);
      e = refresh_fused(n, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
      cp_mlp_destroy(n);
      return api_hip_fail(e, "cp_mlp_create");
    }
    *out = n;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_mlp_create: unexpected exception");
  }
}

void cp_mlp_destroy(cp_mlp* n) {
  if (!n) return;
  free_ws(n);
  for (void* p : {(void*)n->ia, (void*)n->ib, (void*)n->ix, (void*)n->iy, (void*)n->feat,
                  (void*)n->delta, (void*)n->parts})
    if (p) (void)hipFree(p);
  for (float* p : {n->w, n->grad, n->m1, n->m2, n->loss, n->bias_f}) if (p) (void)hipFree(p);
  if (n->wb) (void)hipFree(n->wb);
  if (n->wf) (void)hipFree(n->wf);
  if (n->wbt) (void)hipFree(n->wbt);
  free_train(n);
  if (n->t_parts) (void)hipFree(n->t_parts);
  if (n->d_b_off) (void)hipFree(n->d_b_off);
  if (n->d_width) (void)hipFree(n->d_width);
  delete n;
}

int64_t cp_mlp_num_params(const cp_mlp* n) { return n ? n->n_params : 0; }

int cp_mlp_get_params(const cp_mlp* n, float* d_out, void* stream) {
  if (!n || !d_out) return api_fail(CP_E_ARG, "cp_mlp_get_params: NULL argument");
  hipError_t e = hipMemcpyAsync(d_out, n->w, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_get_params");
}

int cp_mlp_set_params(cp_mlp* n, const float* d_in, void* stream) {
  if (!n || !d_in) return api_fail(CP_E_ARG, "cp_mlp_set_params: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(n->w, d_in, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    refresh_bf16_kernel<<<nblk(n->n_params), 256, 0, st>>>(n->w, n->wb, n->n_params);
    e = hipGetLastError();
    if (e == hipSuccess) e = refresh_fused(n, st);
  }
  return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_set_params");
}

int cp_mlp_get_state(const cp_mlp* n, float* d_m1, float* d_m2, int64_t* step, void* stream) {
  if (!n || !d_m1 || !d_m2) return api_fail(CP_E_ARG, "cp_mlp_get_state: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d_m1, n->m1, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_m2, n->m2, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
  if (step) *step = n->step;
  return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_get_state");
}

int cp_mlp_set_state(cp_mlp* n, const float* d_m1, const float* d_m2, int64_t step, void* stream) {
  if (!n || !d_m1 || !d_m2 || step < 0) return api_fail(CP_E_ARG, "cp_mlp_set_state: bad argument");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(n->m1, d_m1, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(n->m2, d_m2, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) n->step = step;
  return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_set_state");
}

int cp_mlp_forward(cp_mlp* n, int64_t M, const float* d_x, float* d_y, void* stream) {
  try {
    if (!n) return api_fail(CP_E_ARG, "cp_mlp_forward: NULL handle");
    if (M < 0) return api_fail(CP_E_ARG, "cp_mlp_forward: M < 0");
    if (M == 0) return CP_OK;
    if (!d_x || !d_y) return api_fail(CP_E_ARG, "cp_mlp_forward: NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = infer(n, M, d_x, d_y, st);
    return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_forward");
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_mlp_forward: unexpected exception");
  }
}

int cp_mlp_gradients(cp_mlp* n, int64_t M, const float* d_x, const float* d_t, float* d_grad,
                     float* d_loss, void* stream) {
  try {
    if (!n || !d_x || !d_t) return api_fail(CP_E_ARG, "cp_mlp_gradients: NULL argument");
    if (M < 1) return api_fail(CP_E_ARG, "cp_mlp_gradients: M < 1");
    hipStream_t st = (hipStream_t)stream;
    if (n->fusable) {
      hipError_t e = fused_train(n, M, d_x, d_t, 0, n->grad, d_loss, 0.0f, 1.0f, 1.0f, st);
      if (e == hipSuccess && d_grad) e = hipMemcpyAsync(d_grad, n->grad, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
      return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_gradients");
    }
    hipError_t e = forward(n, M, d_x, n->n_in, st);
    if (e == hipSuccess) e = backward(n, M, d_t, st);
    if (e == hipSuccess && d_grad) e = hipMemcpyAsync(d_grad, n->grad, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && d_loss) e = hipMemcpyAsync(d_loss, n->loss, sizeof(float), hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_gradients");
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_mlp_gradients: unexpected exception");
  }
}

int cp_mlp_train_step(cp_mlp* n, int64_t M, const float* d_x, const float* d_t, float lr,
                      float* d_loss, void* stream) {
  try {
    if (!n || !d_x || !d_t) return api_fail(CP_E_ARG, "cp_mlp_train_step: NULL argument");
    if (M < 1 || !(lr > 0)) return api_fail(CP_E_ARG, "cp_mlp_train_step: M < 1 or lr <= 0");
    hipStream_t st = (hipStream_t)stream;
    if (n->fusable) {
      n->step += 1;
      const float c1 = 1.0f - std::pow(0.9f, (float)n->step), c2 = 1.0f - std::pow(0.999f, (float)n->step);
      hipError_t e = fused_train(n, M, d_x, d_t, 1, nullptr, d_loss, lr, c1, c2, st);
      return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_train_step");
    }
    hipError_t e = forward(n, M, d_x, n->n_in, st);
    if (e == hipSuccess) e = backward(n, M, d_t, st);
    if (e != hipSuccess) return api_hip_fail(e, "cp_mlp_train_step");
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)n->step), c2 = 1.0f - std::pow(b2, (float)n->step);
    adam_kernel<<<nblk(n->n_params), 256, 0, st>>>(n->w, n->grad, n->m1, n->m2, n->wb, n->n_params,
                                                    lr, b1, b2, 1e-8f, c1, c2);
    e = hipGetLastError();
    if (e == hipSuccess) e = refresh_fused(n, st);
    if (e == hipSuccess && d_loss) e = hipMemcpyAsync(d_loss, n->loss, sizeof(float), hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_mlp_train_step");
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_mlp_train_step: unexpected exception");
  }
}

int project_motions_warm(const cp_robot* robot, const cp_constraint* constraint,
                         const cp_proj_params* params, cp_mlp* mlp, int32_t n_motions,
                         const float* d_q_from, const float* d_q_to, float* d_xi,
                         int32_t* d_status, int32_t* d_iters, uint64_t* d_work, int32_t flags,
                         void* stream) {
  try {
    if (!robot || !mlp) return api_fail(CP_E_ARG, "project_motions_warm: NULL handle");
    if (n_motions < 0) return api_fail(CP_E_ARG, "project_motions_warm: n_motions < 0");
    cp_proj_params p;
    int rc = api_params(params, &p);
    if (rc != CP_OK) return rc;
    if (p.variant != CP_PROJECT_PARALLEL)
      return api_fail(CP_E_UNSUPPORTED, "project_motions_warm: the warm start serves the parallel projector only");
    ConDev con;
    rc = api_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    const int dof = robot->host.dof;
    if (!dof_supported(dof)) return api_fail(CP_E_UNSUPPORTED, "dof %d", dof);
    if (mlp->n_in != warm_inputs(dof, con.kind) || mlp->n_out != dof)
      return api_fail(CP_E_ARG, "network has %d inputs / %d outputs, the warm start needs %d / %d",
                      mlp->n_in, mlp->n_out, warm_inputs(dof, con.kind), dof);
    if (n_motions == 0) return CP_OK;
    if (!d_q_from || !d_q_to || !d_xi || !d_status) return api_fail(CP_E_ARG, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    const long rows = (long)n_motions * (p.W - 1);
    hipError_t e = hipSuccess;
    if (rows > mlp->warm_rows) {
      if (mlp->feat) (void)hipFree(mlp->feat);
      if (mlp->delta) (void)hipFree(mlp->delta);
      mlp->feat = mlp->delta = nullptr;
      mlp->warm_rows = 0;
      // the fused network computes the features itself
      if (!mlp->fusable) e = hipMalloc((void**)&mlp->feat, sizeof(float) * rows * mlp->n_in);
      if (e == hipSuccess) e = hipMalloc((void**)&mlp->delta, sizeof(float) * rows * dof);
      if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm workspace");
      mlp->warm_rows = rows;
    }
    // constraint parameters as network inputs
    float cp[12] = {0};
    const int n_cp = warm_params(con, cp);
    if (mlp->fusable) {
      e = infer_fused(mlp, warm_feat(robot, con, p.W, d_q_from, d_q_to), rows, mlp->delta, dof, st);
      if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm network");
      return warm_project(robot, con, p, mlp->delta, n_motions, d_q_from, d_q_to, d_xi, d_status,
                          d_iters, d_work, flags, st);
    }
    float* d_cp = mlp->delta;   // borrow the first floats of delta for the parameters
    e = hipMemcpyAsync(d_cp, cp, sizeof(float) * n_cp, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm");
    const unsigned nb = nblk(rows);
    switch (dof) {
      case 2: warm_features_kernel<2><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
      case 3: warm_features_kernel<3><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
      case 6: warm_features_kernel<6><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
      case 7: warm_features_kernel<7><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
      case 9: warm_features_kernel<9><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
      default: warm_features_kernel<14><<<nb, 256, 0, st>>>(robot->dev, p.W, n_motions, d_q_from, d_q_to, d_cp, n_cp, mlp->feat); break;
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = infer(mlp, rows, mlp->feat, mlp->delta, st);
    if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm network");
    return warm_project(robot, con, p, mlp->delta, n_motions, d_q_from, d_q_to, d_xi, d_status,
                        d_iters, d_work, flags, st);
  } catch (...) {
    return api_fail(CP_E_ARG, "project_motions_warm: unexpected exception");
  }
}

int cp_warm_pairs(const cp_robot* robot, const cp_constraint* constraint, int32_t W,
                  int32_t n_motions, const float* d_q_from, const float* d_q_to,
                  const float* d_xi, float* d_x, float* d_t, void* stream) {
  try {
    if (!robot) return api_fail(CP_E_ARG, "cp_warm_pairs: NULL robot");
    if (W < 2 || W > 64 || n_motions < 0) return api_fail(CP_E_ARG, "cp_warm_pairs: W or n_motions out of range");
    ConDev con;
    int rc = api_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    if (n_motions == 0) return CP_OK;
    if (!d_q_from || !d_q_to || !d_xi || !d_x || !d_t) return api_fail(CP_E_ARG, "cp_warm_pairs: NULL buffer");
    const long rows = (long)n_motions * (W - 1);
    const FeatWarm f = warm_feat(robot, con, W, d_q_from, d_q_to);
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = nblk(rows);
    switch (robot->host.dof) {
      case 2: warm_pairs_kernel<2><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      case 3: warm_pairs_kernel<3><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      case 6: warm_pairs_kernel<6><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      case 7: warm_pairs_kernel<7><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      case 9: warm_pairs_kernel<9><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      case 14: warm_pairs_kernel<14><<<nb, 256, 0, st>>>(f, rows, d_xi, d_x, d_t); break;
      default: return api_fail(CP_E_UNSUPPORTED, "dof %d", robot->host.dof);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CP_OK : api_hip_fail(e, "cp_warm_pairs");
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_warm_pairs: unexpected exception");
  }
}

int project_motions_warm_noalloc(const cp_robot* robot, const cp_constraint* constraint,
                                 const cp_proj_params* params, cp_mlp* mlp, int32_t n_motions,
                                 const float* d_q_from, const float* d_q_to, float* d_xi,
                                 int32_t* d_status, int32_t* d_iters, uint64_t* d_work,
                                 int32_t flags, void* stream) {
  try {
    if (!robot || !mlp) return api_fail(CP_E_ARG, "project_motions_warm_noalloc: NULL handle");
    if (n_motions < 0) return api_fail(CP_E_ARG, "project_motions_warm_noalloc: n_motions < 0");
    cp_proj_params p;
    int rc = api_params(params, &p);
    if (rc != CP_OK) return rc;
    if (p.variant != CP_PROJECT_PARALLEL)
      return api_fail(CP_E_UNSUPPORTED, "project_motions_warm_noalloc: the warm start serves the parallel projector only");
    ConDev con;
    rc = api_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    const int dof = robot->host.dof;
    if (!dof_supported(dof)) return api_fail(CP_E_UNSUPPORTED, "dof %d", dof);
    if (mlp->n_in != warm_inputs(dof, con.kind) || mlp->n_out != dof)
      return api_fail(CP_E_ARG, "network has %d inputs / %d outputs, the warm start needs %d / %d",
                      mlp->n_in, mlp->n_out, warm_inputs(dof, con.kind), dof);
    if (!mlp->fusable)
      return api_fail(CP_E_UNSUPPORTED, "project_motions_warm_noalloc: the network's shape needs the "
                      "layer-by-layer path, which allocates (use project_motions_warm)");
    const long rows = (long)n_motions * (p.W - 1);
    if (rows * dof > kNoAllocFloats)
      return api_fail(CP_E_CAPACITY, "project_motions_warm_noalloc: %d motions x %d waypoints x %d joints "
                      "exceed the fixed %ld-float buffer (at most %ld motions here)", n_motions, p.W - 1,
                      dof, kNoAllocFloats, kNoAllocFloats / ((long)(p.W - 1) * dof));
    if (n_motions == 0) return CP_OK;
    if (!d_q_from || !d_q_to || !d_xi || !d_status) return api_fail(CP_E_ARG, "NULL buffer");
    float* delta = nullptr;
    hipError_t e = scratch_address(&delta);
    if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm_noalloc: address of the fixed buffer");
    hipStream_t st = (hipStream_t)stream;
    // every row of delta is written by the network before the projection reads it
    e = infer_fused(mlp, warm_feat(robot, con, p.W, d_q_from, d_q_to), rows, delta, dof, st);
    if (e != hipSuccess) return api_hip_fail(e, "project_motions_warm_noalloc network");
    return warm_project(robot, con, p, delta, n_motions, d_q_from, d_q_to, d_xi, d_status, d_iters,
                        d_work, flags, st);
  } catch (...) {
    return api_fail(CP_E_ARG, "project_motions_warm_noalloc: unexpected exception");
  }
}

}  // extern "C"
