// mlp.hip -- the learned warm start of the source update: a small MLP
// (inputs -> 3 hidden SiLU layers -> outputs) trained on (state, dt) ->
// (post-update T_gas, E_g) pairs produced by the FP64 solver, used to give the
// Newton iteration its initial guess.  Plain Newton from the old state stays
// the fallback and decides the result (the solver converges to the same root
// whatever the guess).
//
// All tensors are FP32 in HBM; every matrix product runs on the gfx950 matrix
// cores as BF16 x BF16 -> FP32 (v_mfma_f32_16x16x32_bf16): operands are
// rounded to BF16 when a 64x32 / 32x64 tile is staged in LDS, accumulation is
// FP32.  Master weights and Adam moments are FP32.
//
// Lane layout of v_mfma_f32_16x16x32_bf16 used below (checked by the GPU
// tests against a reference product): lane l holds A[l%16][8(l/16) .. +7],
// B[8(l/16) .. +7][l%16], and accumulators C[4(l/16) .. +3][l%16].
#include <hip/hip_runtime.h>

#include <mutex>

#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/mgrhd.h"
#include "batch_infer.hpp"
#include "planck_device.hpp"

namespace mgrhd {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDK = BK + 8;  // LDS row pitch in bf16 (80 bytes: 16-byte aligned, skewed banks)

enum Epi : int { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_ATOMIC = 3 };

// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) (SiLU, keeping the
// pre-activation in Z).  op(A) = A (row-major, lda) or A^T (A stored K x M);
// op(B) = B (row-major K x N, ldb) or B^T (B stored N x K).
// F32: operands kept in FP32 and multiplied by v_mfma_f32_16x16x4_f32 (lane l
// holds A[l%16][l/16] and B[l/16][l%16] of a 4-deep slice; same accumulator
// layout), the checking path of the network's products.
template <bool TA, bool TB, int EPI, bool F32 = false>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb,
                                              const float* __restrict__ bias, float* __restrict__ C,
                                              int ldc, float* __restrict__ Z, int64_t M, int N,
                                              int K) {
  using OpT = typename std::conditional<F32, float, __bf16>::type;
  __shared__ __attribute__((aligned(16))) OpT As[BM][LDK];
  __shared__ __attribute__((aligned(16))) OpT Bs[BN][LDK];
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  // split-K (EPI_ATOMIC): block z reduces K range [z Kc, (z+1) Kc) and adds into C
  const int Kc = (EPI == EPI_ATOMIC) ? (((K + gridDim.z - 1) / gridDim.z + BK - 1) / BK) * BK : K;
  const int kbeg = (EPI == EPI_ATOMIC) ? (int)blockIdx.z * Kc : 0;
  const int kend = (EPI == EPI_ATOMIC) ? min(K, kbeg + Kc) : K;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // stage A tile (BM x BK) and B tile (BK x BN) as bf16, k contiguous
#pragma unroll
    for (int r = 0; r < (BM * BK) / 256; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (TA) {  // coalesced along m
        mm = e % BM;
        kk = e / BM;
      } else {   // coalesced along k
        kk = e % BK;
        mm = e / BK;
      }
      const int64_t gm = m0 + mm;
      const int gk = k0 + kk;
      float x = 0.f;
      if (gm < M && gk < kend) x = TA ? A[(int64_t)gk * lda + gm] : A[gm * lda + gk];
      As[mm][kk] = (OpT)x;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / 256; ++r) {
      const int e = tid + 256 * r;
      int nn, kk;
      if (TB) {  // B stored N x K: coalesced along k
        kk = e % BK;
        nn = e / BK;
      } else {   // B stored K x N: coalesced along n
        nn = e % BN;
        kk = e / BN;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      float x = 0.f;
      if (gn < N && gk < kend) x = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[nn][kk] = (OpT)x;
    }
    __syncthreads();
    const int r16 = lane % 16;
    if constexpr (F32) {
      const int k4 = lane / 16;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = As[wm + 16 * a + r16][kk + k4];
#pragma unroll
        for (int b = 0; b < 2; ++b) bfr[b] = Bs[wn + 16 * b + r16][kk + k4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bfr[b], acc[a][b], 0, 0, 0);
      }
    } else {
      const int kq = 8 * (lane / 16);
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = *(const bf16x8*)&As[wm + 16 * a + r16][kq];
#pragma unroll
      for (int b = 0; b < 2; ++b) bfr[b] = *(const bf16x8*)&Bs[wn + 16 * b + r16][kq];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: lane holds C[4(l/16)+i][l%16] of each 16x16 tile
  const int col16 = lane % 16, row4 = 4 * (lane / 16);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + wn + 16 * b + col16;
      if (n >= N) continue;
      const float bv = (EPI == EPI_BIAS || EPI == EPI_BIAS_SILU) ? bias[n] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + wm + 16 * a + row4 + i;
        if (m >= M) continue;
        float z = acc[a][b][i] + bv;
        if (EPI == EPI_BIAS_SILU) {
          if (Z) Z[m * ldc + n] = z;  // pre-activation, kept for the backward pass
          z = z / (1.f + expf(-z));
        }
        if (EPI == EPI_ATOMIC)
          atomicAdd(&C[m * ldc + n], z);
        else
          C[m * ldc + n] = z;
      }
    }
}

// dZ = dH * SiLU'(Z), SiLU'(z) = s (1 + z (1 - s)), s = 1/(1+e^-z)
__global__ void k_silu_bwd(const float* __restrict__ dH, const float* __restrict__ Z,
                           float* __restrict__ dZ, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float z = Z[i];
    const float s = 1.f / (1.f + expf(-z));
    dZ[i] = dH[i] * (s * (1.f + z * (1.f - s)));
  }
}

// column sums of a row-major [rows x N] matrix (bias gradients) added into
// out (cleared before): block b sums rows [256 b, 256 b + 256), thread n
// column n (N <= 256)
__global__ void k_colsum(const float* __restrict__ X, int64_t rows, int N, float* __restrict__ out) {
  const int n = threadIdx.x;
  if (n >= N) return;
  const int64_t r0 = (int64_t)blockIdx.x * 256, r1 = min(rows, r0 + 256);
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) s += X[r * N + n];
  atomicAdd(&out[n], s);
}

// mean-squared error: dY = 2 (Y - T) / (rows * N), loss = mean (Y - T)^2
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                      float scale, float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float part[256];
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d * scale;
    acc += d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, part[0] * scale);
}

__global__ void k_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// Adam on FP32 master parameters
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// Physics side: features, targets and the Newton guess (FP64 state).
//
// Features per cell (2 + 3 N_g), stored feature-major X[f * n + i]:
//   ln T, ln rho, ln(E_g / a T^4) (clamped to [-50, 50]), |F_g| / (c E_g)
//   (clamped to [0, 2]), ln(c_hat dt chi_0E,g) (PPL-fixed mean of the group),
// each z-scored with the training statistics (mean, inv_std).
// Targets per cell (1 + N_g), row-major Y[i * (1+N_g) + o]:
//   ln(T_new / T), ln(E_g,new / a T^4) (clamped to [-50, 50]).
struct PhysArgs {
  const double* E;
  const double* F;
  const double* rho;
  const double* egas;
  const double* v;
  const double* kappa;
  const double* edges;
  const double* chi_lo;
  const double* alpha;
  int64_t n;
  int32_t ng;
  int32_t pad;
  double dt, chat, c, a, cv;
};

__device__ __forceinline__ double cell_T(const PhysArgs& p, int64_t i) {
  const int64_t n = p.n;
  const double v0 = p.v[i], v1 = p.v[n + i], v2 = p.v[2 * n + i];
  const double rho = p.rho[i];
  return (p.egas[i] - 0.5 * rho * (v0 * v0 + v1 * v1 + v2 * v2)) / (rho * p.cv);
}

__global__ void k_features(PhysArgs p, const float* __restrict__ mean,
                           const float* __restrict__ istd, float* __restrict__ X) {
  // ln(chi_0E,g per unit rho kappa) of the PPL-fixed group mean, per group
  __shared__ double lchi[MGRHD_MAX_GROUPS];
  const int ng = p.ng;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    const double L = log(p.edges[g + 1] / p.edges[g]);
    const double ac = p.alpha ? p.alpha[g] : 0.0;
    lchi[g] = log(p.chi_lo[g] * mean_ratio(ac, -1.0, L));
  }
  __syncthreads();
  const int64_t n = p.n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double T = fmax(cell_T(p, i), 1e-300);
    const double rho = p.rho[i];
    const double aT4 = p.a * (T * T) * (T * T);
    const double kap = p.kappa ? p.kappa[i] : 1.0;
    const double lcell = log(p.chat * p.dt * rho * kap);
    auto put = [&](int f, double x) { X[(int64_t)f * n + i] = (float)((x - mean[f]) * istd[f]); };
    put(0, log(T));
    put(1, log(rho));
    for (int g = 0; g < ng; ++g) {
      const double E = p.E[(int64_t)g * n + i];
      const double f0 = p.F[((int64_t)0 * ng + g) * n + i];
      const double f1 = p.F[((int64_t)1 * ng + g) * n + i];
      const double f2 = p.F[((int64_t)2 * ng + g) * n + i];
      const double le = E > 0.0 ? fmin(fmax(log(E / aT4), -50.0), 50.0) : -50.0;
      const double fr = E > 0.0 ? fmin(sqrt(f0 * f0 + f1 * f1 + f2 * f2) / (p.c * E), 2.0) : 0.0;
      put(2 + g, le);
      put(2 + ng + g, fr);
      put(2 + 2 * ng + g, lcell + lchi[g]);
    }
  }
}

// targets from the state before (p) and after (E_new, egas_new, v_new) the update
__global__ void k_targets(PhysArgs p, const double* __restrict__ E_new,
                          const double* __restrict__ egas_new, const double* __restrict__ v_new,
                          float* __restrict__ Y) {
  const int64_t n = p.n;
  const int ng = p.ng, no = ng + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double T = fmax(cell_T(p, i), 1e-300);
    const double aT4 = p.a * (T * T) * (T * T);
    const double w0 = v_new[i], w1 = v_new[n + i], w2 = v_new[2 * n + i];
    const double rho = p.rho[i];
    const double Tn = (egas_new[i] - 0.5 * rho * (w0 * w0 + w1 * w1 + w2 * w2)) / (rho * p.cv);
    Y[i * no] = (float)(Tn > 0.0 ? log(Tn / T) : 0.0);
    for (int g = 0; g < ng; ++g) {
      const double E = E_new[(int64_t)g * n + i];
      Y[i * no + 1 + g] = (float)(E > 0.0 ? fmin(fmax(log(E / aT4), -50.0), 50.0) : -50.0);
    }
  }
}

// Newton guess from the de-normalised prediction: (E_gas, R_g), or E_gas alone
// (kind 1; the solver then takes each R_g from its group balance).
__global__ void k_guess(PhysArgs p, const float* __restrict__ Yn, const float* __restrict__ ymean,
                        const float* __restrict__ ystd, const double* __restrict__ S,
                        int kind, double* __restrict__ guess) {
  const int64_t n = p.n;
  const int ng = p.ng, no = ng + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double T = fmax(cell_T(p, i), 1e-300);
    const double aT4 = p.a * (T * T) * (T * T);
    const double v0 = p.v[i], v1 = p.v[n + i], v2 = p.v[2 * n + i];
    const double rho = p.rho[i];
    const double yT = (double)Yn[i * no] * ystd[0] + ymean[0];
    const double Tg = T * exp(fmin(fmax(yT, -5.0), 5.0));
    guess[i] = rho * p.cv * Tg + 0.5 * rho * (v0 * v0 + v1 * v1 + v2 * v2);
    if (kind == 1) continue;
    for (int g = 0; g < ng; ++g) {
      const double yE = (double)Yn[i * no + 1 + g] * ystd[1 + g] + ymean[1 + g];
      const double Eg = aT4 * exp(fmin(fmax(yE, -60.0), 60.0));
      const double sg = S ? S[(int64_t)g * n + i] : 0.0;
      guess[(int64_t)(g + 1) * n + i] = Eg - p.E[(int64_t)g * n + i] - sg;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused inference: features -> 3 SiLU layers -> output -> Newton guess, one
// tile of kTile cells per block iteration, activations kept in LDS as BF16.
// Weights are BF16 copies [N_pad x K_pad] (zero padded) read straight from
// L2 as matrix-core B fragments; wave w computes n-tiles w, w+4, ... for all
// four 16-row tiles, so every weight element is read once per cell tile.
// Features are formed in FP32 (they are rounded to BF16 for the products).
constexpr int kTile = 64;
constexpr int kHidden = 128;               // hidden width of the fused path
constexpr int kHPad = kHidden + 8;         // LDS row pitch of a hidden tile
constexpr int kMaxKin = 416;               // padded input width (N_g <= 138)

struct InferArgs {
  PhysArgs p;
  const float* xmean;
  const float* xistd;
  const float* ymean;
  const float* ystd;
  const __bf16* W[4];  // [N_pad x K_pad] each
  const float* b[4];   // [N_pad] each (zero padded)
  int K_pad[4], N_pad[4];
  int n_in, n_out, kind;
  const double* S;
  double* guess;
};

// one layer: out = act(in W^T + b) on a kTile-row tile; in: LDS bf16 rows of
// pitch ldi; hidden layers write bf16 to `hout` (pitch kHPad), the output
// layer writes fp32 to `fout` (pitch ldo).
template <bool HIDDEN>
__device__ __forceinline__ void tile_layer(const __bf16* in, int ldi, const __bf16* __restrict__ W,
                                           const float* __restrict__ bias, int K_pad, int n_tiles,
                                           __bf16* hout, float* fout, int ldo) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int r16 = lane % 16, kq = 8 * (lane / 16);
  for (int nt0 = wave; nt0 < n_tiles; nt0 += 8) {
    // this wave's n-tiles: nt0 and nt0 + 4 (when present)
    const int nts[2] = {nt0, nt0 + 4};
    const bool two = nt0 + 4 < n_tiles;
    floatx4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[a][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const __bf16* w0 = W + (int64_t)(16 * nts[0] + r16) * K_pad + kq;
    const __bf16* w1 = W + (int64_t)(16 * (two ? nts[1] : nts[0]) + r16) * K_pad + kq;
    const int ksteps = K_pad / 32;
    // the B fragments of up to kPre k-steps are requested at once (one L2
    // latency per layer instead of one per k-step)
    constexpr int kPre = 4;
    for (int kb = 0; kb < ksteps; kb += kPre) {
      bf16x8 bfr[kPre][2];
#pragma unroll
      for (int kk = 0; kk < kPre; ++kk) {
        if (kb + kk < ksteps) {
          bfr[kk][0] = *(const bf16x8*)(w0 + 32 * (kb + kk));
          bfr[kk][1] = *(const bf16x8*)(w1 + 32 * (kb + kk));
        }
      }
#pragma unroll
      for (int kk = 0; kk < kPre; ++kk) {
        if (kb + kk >= ksteps) break;
        const int k0 = 32 * (kb + kk);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const bf16x8 af = *(const bf16x8*)(in + (16 * a + r16) * ldi + k0 + kq);
          acc[a][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[kk][0], acc[a][0], 0, 0, 0);
          if (two)
            acc[a][1] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[kk][1], acc[a][1], 0, 0, 0);
        }
      }
    }
    const int col16 = lane % 16, row4 = 4 * (lane / 16);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t == 1 && !two) break;
      const int n = 16 * nts[t] + col16;
      const float bv = bias[n];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * a + row4 + i;
          float z = acc[a][t][i] + bv;
          if (HIDDEN) {
            z = z / (1.f + __expf(-z));
            hout[r * kHPad + n] = (__bf16)z;
          } else {
            fout[r * ldo + n] = z;
          }
        }
    }
  }
}

// log of each group's PPL-fixed mean opacity per unit rho kappa (a feature
// of the network), into LDS; the caller synchronises.
__device__ __forceinline__ void infer_lchi(const PhysArgs& p, float* lchi) {
  for (int g = threadIdx.x; g < p.ng; g += blockDim.x) {
    const double L = log(p.edges[g + 1] / p.edges[g]);
    const double ac = p.alpha ? p.alpha[g] : 0.0;
    lchi[g] = (float)log(p.chi_lo[g] * mean_ratio(ac, -1.0, L));
  }
}

// The fused inference of the cells [i0, min(i0 + kTile, i1)) of one state:
// features, the three hidden layers and the output on the matrix cores, and
// the Newton guess written to `guess` (kind 1: [n]; kind 0: [N_g+1][n]).
// Every thread of the workgroup calls it (it synchronises); smem is the
// dynamic LDS of k_infer, lchi that state's feature table.
__device__ __forceinline__ void infer_tile(const InferArgs& q, const PhysArgs& p, double* guess,
                                           const double* S, const float* lchi, const float* xs,
                                           int64_t i0, int64_t i1, unsigned char* smem) {
  const int ng = p.ng;
  const int64_t n = p.n;
  const int ldx = q.K_pad[0] + 8;
  __bf16* X = (__bf16*)smem;                                  // [kTile][ldx]; later H_b / out
  __bf16* Ha = X + kTile * (ldx > kHPad ? ldx : kHPad);       // [kTile][kHPad]
  const int r = threadIdx.x / 4, qd = threadIdx.x % 4;
  const int64_t i = i0 + r;
  const bool live = i < i1;
  // the cell's temperature, density and kinetic energy, kept for the guess
  double Tc = 1.0, rh = 1.0, ke = 0.0;
  // ---- features (normalised, bf16) ----
  {
    float T = 1.f, rho = 1.f, lcell = 0.f;
    double iaT4 = 1.0;  // 1/(a T^4)
    if (live) {
      const double v0 = p.v[i], v1 = p.v[n + i], v2 = p.v[2 * n + i];
      rh = p.rho[i];
      ke = 0.5 * rh * (v0 * v0 + v1 * v1 + v2 * v2);
      Tc = fmax((p.egas[i] - ke) / (rh * p.cv), 1e-300);
      const double kap = p.kappa ? p.kappa[i] : 1.0;
      T = (float)Tc;
      rho = (float)rh;
      iaT4 = 1.0 / (p.a * (Tc * Tc) * (Tc * Tc));
      lcell = (float)log(p.chat * p.dt * rh * kap);
    }
    __bf16* xr = X + r * ldx;
    // xs: the input statistics in LDS, mean [K_pad] then 1/std [K_pad]
    auto put = [&](int f, float x) { xr[f] = (__bf16)((x - xs[f]) * xs[q.K_pad[0] + f]); };
    if (qd == 0) {
      put(0, live ? __logf(T) : 0.f);
      put(1, live ? __logf(rho) : 0.f);
    }
    // sixteen groups per chunk: their 64 loads are in flight together (all of
    // a thread's loads at 64 groups)
    constexpr int kU = 16;
    for (int g0 = qd; g0 < ng; g0 += 4 * kU) {
      double E[kU], f0[kU], f1[kU], f2[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int g = g0 + 4 * u;
        E[u] = f0[u] = f1[u] = f2[u] = 0.0;
        if (live && g < ng) {
          E[u] = p.E[(int64_t)g * n + i];
          f0[u] = p.F[((int64_t)0 * ng + g) * n + i];
          f1[u] = p.F[((int64_t)1 * ng + g) * n + i];
          f2[u] = p.F[((int64_t)2 * ng + g) * n + i];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int g = g0 + 4 * u;
        if (g >= ng) break;
        float le = -50.f, fr = 0.f;
        if (E[u] > 0.0) {
          // E / (a T^4) rounded to FP32: beyond its range the logarithm is
          // past the clamp at +-50 either way
          le = fminf(fmaxf(__logf((float)(E[u] * iaT4)), -50.f), 50.f);
          fr = fminf((float)(sqrt(f0[u] * f0[u] + f1[u] * f1[u] + f2[u] * f2[u]) /
                             (p.c * E[u])), 2.f);
        }
        put(2 + g, le);
        put(2 + ng + g, fr);
        put(2 + 2 * ng + g, lcell + lchi[g]);
      }
    }
    for (int f = q.n_in + qd; f < q.K_pad[0]; f += 4) xr[f] = (__bf16)0.f;
  }
  __syncthreads();
  // ---- layers: X -> Ha -> Hb (in X's space) -> Ha -> out (fp32 in X's space) ----
  __bf16* Hb = X;
  tile_layer<true>(X, ldx, q.W[0], q.b[0], q.K_pad[0], q.N_pad[0] / 16, Ha, nullptr, 0);
  __syncthreads();
  tile_layer<true>(Ha, kHPad, q.W[1], q.b[1], q.K_pad[1], q.N_pad[1] / 16, Hb, nullptr, 0);
  __syncthreads();
  tile_layer<true>(Hb, kHPad, q.W[2], q.b[2], q.K_pad[2], q.N_pad[2] / 16, Ha, nullptr, 0);
  __syncthreads();
  float* out = (float*)X;
  const int ldo = q.N_pad[3];
  const int out_tiles = q.kind == 1 ? 1 : q.N_pad[3] / 16;
  tile_layer<false>(Ha, kHPad, q.W[3], q.b[3], q.K_pad[3], out_tiles, nullptr, out, ldo);
  __syncthreads();
  // ---- Newton guess ----
  if (live) {
    const float* o = out + r * ldo;
    if (qd == 0) {
      const double yT = (double)o[0] * q.ystd[0] + q.ymean[0];
      guess[i] = rh * p.cv * Tc * exp(fmin(fmax(yT, -5.0), 5.0)) + ke;
    }
    if (q.kind == 0) {
      const double aT4 = p.a * (Tc * Tc) * (Tc * Tc);
      for (int g = qd; g < ng; g += 4) {
        const double yE = (double)o[1 + g] * q.ystd[1 + g] + q.ymean[1 + g];
        const double sg = S ? S[(int64_t)g * n + i] : 0.0;
        guess[(int64_t)(g + 1) * n + i] =
            aT4 * exp(fmin(fmax(yE, -60.0), 60.0)) - p.E[(int64_t)g * n + i] - sg;
      }
    }
  }
  __syncthreads();
}

// LDS of the fused inference: the input tile (or a hidden tile), a hidden
// tile, the feature table of N_g floats and the input statistics (2 K_pad
// floats, after the table at a K_pad-float offset: N_g <= K_pad).
__host__ __device__ inline size_t infer_lds_bytes(int k_pad0, int ng) {
  const int ldx = k_pad0 + 8;
  (void)ng;
  return sizeof(__bf16) * (size_t)kTile * ((ldx > kHPad ? ldx : kHPad) + kHPad) +
         sizeof(float) * 3 * (size_t)k_pad0;
}

// The input statistics into LDS (mean, then 1/std; zero beyond n_in).
__device__ __forceinline__ void infer_stats(const InferArgs& q, float* xs) {
  for (int f = threadIdx.x; f < q.K_pad[0]; f += blockDim.x) {
    xs[f] = f < q.n_in ? q.xmean[f] : 0.f;
    xs[q.K_pad[0] + f] = f < q.n_in ? q.xistd[f] : 0.f;
  }
}

__global__ __launch_bounds__(256, 2) void k_infer(InferArgs q) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const PhysArgs& p = q.p;
  const int ldx = q.K_pad[0] + 8;
  float* lchi = (float*)(smem + sizeof(__bf16) * (size_t)kTile *
                                    ((ldx > kHPad ? ldx : kHPad) + kHPad));
  float* xs = lchi + q.K_pad[0];
  infer_lchi(p, lchi);
  infer_stats(q, xs);
  __syncthreads();
  const int64_t tiles = (p.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x)
    infer_tile(q, p, q.guess, q.S, lchi, xs, tile * kTile, p.n, smem);
}

// The fused inference over the work items [lo, hi) of a batch of patches
// (one group count): each workgroup takes items in turn, rebuilds the
// feature table when the patch changes, and infers the item's cells tile by
// tile into that patch's guess buffer.
struct InferItemsArgs {
  InferArgs q;          // weights, statistics, kind (q.p, q.guess, q.S unused)
  const KArgs* patches;
  const BatchItem* items;
  int64_t lo, hi;
};

__global__ __launch_bounds__(256, 2) void k_infer_items(InferItemsArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int ldx = a.q.K_pad[0] + 8;
  float* lchi = (float*)(smem + sizeof(__bf16) * (size_t)kTile *
                                    ((ldx > kHPad ? ldx : kHPad) + kHPad));
  float* xs = lchi + a.q.K_pad[0];
  infer_stats(a.q, xs);  // (published by the first patch's barrier below)
  int cur = -1;
  for (int64_t it = a.lo + blockIdx.x; it < a.hi; it += gridDim.x) {
    const BatchItem item = a.items[it];
    const KArgs& k = a.patches[item.patch];
    PhysArgs p;
    p.E = k.E;
    p.F = k.F;
    p.rho = k.rho;
    p.egas = k.egas;
    p.v = k.v;
    p.kappa = k.kappa;
    p.edges = k.edges;
    p.chi_lo = k.chi_lo;
    p.alpha = k.alpha;
    p.n = k.n;
    p.ng = k.ng;
    p.pad = 0;
    p.dt = k.dt;
    p.chat = k.chat;
    p.c = k.c;
    p.a = k.a;
    p.cv = k.cv;
    if (item.patch != cur) {  // uniform over the workgroup
      __syncthreads();        // the previous patch's table is no longer read
      infer_lchi(p, lchi);
      __syncthreads();
      cur = item.patch;
    }
    double* guess = const_cast<double*>(k.guess);  // the batch's guess buffer
    for (int64_t i0 = item.c0; i0 < item.c1; i0 += kTile)
      infer_tile(a.q, p, guess, k.S, lchi, xs, i0, item.c1, smem);
  }
}

// fp32 weights [N x K] -> bf16 [N_pad x K_pad] (zero padded); biases -> fp32 [N_pad]
__global__ void k_pack(const float* __restrict__ W, const float* __restrict__ b, int N, int K,
                       int N_pad, int K_pad, __bf16* __restrict__ Wp, float* __restrict__ bp) {
  const int64_t total = (int64_t)N_pad * K_pad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int nn = (int)(e / K_pad), kk = (int)(e % K_pad);
    Wp[e] = (__bf16)((nn < N && kk < K) ? W[(int64_t)nn * K + kk] : 0.f);
    if (kk == 0) bp[nn] = nn < N ? b[nn] : 0.f;
  }
}

}  // namespace mlp
}  // namespace mgrhd

using namespace mgrhd::mlp;

// ---------------------------------------------------------------------------
// The network handle: layer sizes, FP32 master parameters, gradients, Adam
// moments and activation scratch for up to max_rows rows per call.
struct mgrhd_mlp {
  int n_in = 0, n_hidden = 0, n_out = 0;
  static constexpr int kLayers = 4;  // 3 hidden SiLU layers + linear output
  int64_t max_rows = 0;
  int64_t n_params = 0;
  int in_dim[kLayers], out_dim[kLayers];
  int64_t w_off[kLayers], b_off[kLayers];
  float* params = nullptr;  // [n_params] weights (out x in, row-major) then biases
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* act = nullptr;     // H1..H3, Z1..Z3, Y, dY, dH, dZ scratch
  float* loss = nullptr;    // device scalar
  int64_t step = 0;
  float* H[3];
  float* Zs[3];
  float* Y = nullptr;
  float* dY = nullptr;
  float* dA = nullptr;
  float* dB = nullptr;
  // BF16 copies for the fused inference (repacked when the weights change)
  __bf16* wpack = nullptr;
  float* bpack = nullptr;
  int k_pad[kLayers], n_pad[kLayers];
  int64_t wp_off[kLayers], bp_off[kLayers];
  bool dirty = true;
  bool fp32 = false;  // FP32 operands in the forward and backward products
};

static inline dim3 grid1(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65535 * 4) b = 65535 * 4;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

template <bool TA, bool TB, int EPI>
static void gemm(hipStream_t s, const float* A, int lda, const float* B, int ldb, const float* bias,
                 float* C, int ldc, float* Z, int64_t M, int N, int K, int splits = 1,
                 bool f32 = false) {
  dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)splits);
  if (f32)
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI, true>), grid, dim3(256), 0, s, A, lda, B, ldb, bias,
                       C, ldc, Z, M, N, K);
  else
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI, false>), grid, dim3(256), 0, s, A, lda, B, ldb, bias,
                       C, ldc, Z, M, N, K);
}

// forward of `rows` rows.  X_fm: features feature-major [n_in x ld_x]; the
// rows are X_fm[:, 0:rows].  Output Y row-major [rows x n_out].
static void forward(mgrhd_mlp* m, hipStream_t s, const float* X_fm, int64_t ld_x, int64_t rows,
                    float* Y, bool keep_z) {
  const float* in = X_fm;
  for (int l = 0; l < 3; ++l) {
    const float* W = m->params + m->w_off[l];
    const float* b = m->params + m->b_off[l];
    if (l == 0)
      gemm<true, true, EPI_BIAS_SILU>(s, in, (int)ld_x, W, m->in_dim[l], b, m->H[l],
                                      m->out_dim[l], keep_z ? m->Zs[l] : nullptr, rows,
                                      m->out_dim[l], m->in_dim[l], 1, m->fp32);
    else
      gemm<false, true, EPI_BIAS_SILU>(s, in, m->in_dim[l], W, m->in_dim[l], b, m->H[l],
                                       m->out_dim[l], keep_z ? m->Zs[l] : nullptr, rows,
                                       m->out_dim[l], m->in_dim[l], 1, m->fp32);
    in = m->H[l];
  }
  gemm<false, true, EPI_BIAS>(s, in, m->in_dim[3], m->params + m->w_off[3], m->in_dim[3],
                              m->params + m->b_off[3], Y, m->out_dim[3], nullptr, rows,
                              m->out_dim[3], m->in_dim[3], 1, m->fp32);
}

// backward: gradients of mean((Y - T)^2) with respect to all parameters
static void backward(mgrhd_mlp* m, hipStream_t s, const float* X_fm, int64_t ld_x, int64_t rows,
                     const float* Tgt) {
  const int64_t ny = rows * m->n_out;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, m->loss, (int64_t)1);
  hipLaunchKernelGGL(k_mse, grid1(ny), dim3(256), 0, s, m->Y, Tgt, ny, 1.f / (float)ny, m->dY,
                     m->loss);
  // the weight and bias gradients are accumulated (split over rows): clear them
  hipLaunchKernelGGL(k_zero, grid1(m->n_params), dim3(256), 0, s, m->grads, m->n_params);
  // rows per split of the weight-gradient products: enough blocks to fill the chip
  const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(64, rows / 256));
  const float* dOut = m->dY;  // gradient w.r.t. the current layer's output (pre-activation for l=3)
  for (int l = 3; l >= 0; --l) {
    const int no = m->out_dim[l], ni = m->in_dim[l];
    float* dW = m->grads + m->w_off[l];
    float* db = m->grads + m->b_off[l];
    // dW = dOut^T [no x rows] . input [rows x ni]
    if (l == 0)  // input X feature-major: op(B) = (X_fm)^T, stored ni x ld_x
      gemm<true, true, EPI_ATOMIC>(s, dOut, no, X_fm, (int)ld_x, nullptr, dW, ni, nullptr, no,
                                   ni, (int)rows, splits, m->fp32);
    else
      gemm<true, false, EPI_ATOMIC>(s, dOut, no, m->H[l - 1], ni, nullptr, dW, ni, nullptr, no,
                                    ni, (int)rows, splits, m->fp32);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, dOut,
                       rows, no, db);
    if (l == 0) break;
    // dH_{l-1} = dOut [rows x no] . W_l [no x ni]; then through SiLU
    float* dH = m->dA;
    gemm<false, false, EPI_NONE>(s, dOut, no, m->params + m->w_off[l], ni, nullptr, dH, ni,
                                 nullptr, rows, ni, no, 1, m->fp32);
    float* dZ = (dOut == m->dB) ? m->dA : m->dB;
    if (dZ == dH) dZ = m->dB;
    hipLaunchKernelGGL(k_silu_bwd, grid1(rows * ni), dim3(256), 0, s, dH, m->Zs[l - 1], dZ,
                       rows * (int64_t)ni);
    dOut = dZ;
  }
}

extern "C" {

int mgrhd_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t max_rows,
                     uint64_t seed, mgrhd_mlp** out) {
  if (!out) return MGRHD_E_NULL;
  *out = nullptr;
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || max_rows < 1) return MGRHD_E_SIZE;
  if (n_hidden > 256 || n_out > 256) return MGRHD_E_SIZE;  // bias-gradient kernel width
  mgrhd_mlp* m = new (std::nothrow) mgrhd_mlp();
  if (!m) return MGRHD_E_DEVICE;
  m->n_in = n_in;
  m->n_hidden = n_hidden;
  m->n_out = n_out;
  m->max_rows = max_rows;
  const int dims[5] = {n_in, n_hidden, n_hidden, n_hidden, n_out};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    m->in_dim[l] = dims[l];
    m->out_dim[l] = dims[l + 1];
    m->w_off[l] = off;
    off += (int64_t)dims[l] * dims[l + 1];
  }
  for (int l = 0; l < 4; ++l) {
    m->b_off[l] = off;
    off += dims[l + 1];
  }
  m->n_params = off;
  // He-uniform weights for SiLU layers, zero biases (host-side init, seeded)
  std::vector<float> h(off, 0.f);
  uint64_t z = seed ? seed : 0x9E3779B97F4A7C15ULL;
  auto next = [&]() {
    z += 0x9E3779B97F4A7C15ULL;
    uint64_t x = z;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1.0p-53;
  };
  for (int l = 0; l < 4; ++l) {
    const double lim = std::sqrt(6.0 / dims[l]) * (l == 3 ? 0.5 : 1.0);
    for (int64_t k = 0; k < (int64_t)dims[l] * dims[l + 1]; ++k)
      h[m->w_off[l] + k] = (float)((2.0 * next() - 1.0) * lim);
  }
  const int64_t act = (int64_t)max_rows * (6 * n_hidden + 2 * n_out + 2 * std::max(n_hidden, n_out));
  int64_t wtot = 0, btot = 0;
  for (int l = 0; l < 4; ++l) {
    m->k_pad[l] = (dims[l] + 31) / 32 * 32;
    m->n_pad[l] = (dims[l + 1] + 15) / 16 * 16;
    m->wp_off[l] = wtot;
    m->bp_off[l] = btot;
    wtot += (int64_t)m->k_pad[l] * m->n_pad[l];
    btot += m->n_pad[l];
  }
  bool ok = hipMalloc(&m->wpack, sizeof(__bf16) * wtot) == hipSuccess &&
            hipMalloc(&m->bpack, sizeof(float) * btot) == hipSuccess &&
            hipMalloc(&m->params, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&m->grads, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&m->adam_m, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&m->adam_v, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&m->act, sizeof(float) * act) == hipSuccess &&
            hipMalloc(&m->loss, sizeof(float)) == hipSuccess;
  if (ok) {
    ok = hipMemcpy(m->params, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) == hipSuccess;
    std::vector<float> zero(off, 0.f);
    ok = ok && hipMemcpy(m->adam_m, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
                   hipSuccess;
    ok = ok && hipMemcpy(m->adam_v, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
                   hipSuccess;
    ok = ok && hipMemcpy(m->grads, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
                   hipSuccess;
  }
  if (!ok) {
    mgrhd_mlp_destroy(m);
    return MGRHD_E_DEVICE;
  }
  float* p = m->act;
  for (int l = 0; l < 3; ++l) {
    m->H[l] = p;
    p += max_rows * n_hidden;
    m->Zs[l] = p;
    p += max_rows * n_hidden;
  }
  m->Y = p;
  p += max_rows * n_out;
  m->dY = p;
  p += max_rows * n_out;
  const int w = std::max(n_hidden, n_out);
  m->dA = p;
  p += max_rows * w;
  m->dB = p;
  *out = m;
  return 0;
}

int64_t mgrhd_mlp_num_params(const mgrhd_mlp* m) { return m ? m->n_params : -1; }

int mgrhd_mlp_get_params(const mgrhd_mlp* m, float* host, int32_t which) {
  if (!m || !host) return MGRHD_E_NULL;
  const float* src = which == 0 ? m->params : which == 1 ? m->grads : nullptr;
  if (!src) return MGRHD_E_OPTION;
  return hipMemcpy(host, src, sizeof(float) * m->n_params, hipMemcpyDeviceToHost) == hipSuccess
             ? 0 : MGRHD_E_DEVICE;
}

int mgrhd_mlp_set_params(mgrhd_mlp* m, const float* host) {
  if (!m || !host) return MGRHD_E_NULL;
  m->dirty = true;
  return hipMemcpy(m->params, host, sizeof(float) * m->n_params, hipMemcpyHostToDevice) ==
                 hipSuccess
             ? 0 : MGRHD_E_DEVICE;
}

// File layout: 8-byte magic "MGRHDMLP", int32 version (1), int32 n_in,
// n_hidden, n_out, int64 n_params, then n_params float32 parameters (the
// order of mgrhd_mlp_get_params), little-endian as the host writes them.
static const char kMlpMagic[8] = {'M', 'G', 'R', 'H', 'D', 'M', 'L', 'P'};

int mgrhd_mlp_save(const mgrhd_mlp* m, const char* path) {
  if (!m || !path) return MGRHD_E_NULL;
  std::vector<float> p((size_t)m->n_params);
  if (hipMemcpy(p.data(), m->params, sizeof(float) * p.size(), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return MGRHD_E_DEVICE;
  FILE* f = std::fopen(path, "wb");
  if (!f) return MGRHD_E_OPTION;
  const int32_t head[4] = {1, m->n_in, m->n_hidden, m->n_out};
  const int64_t np = m->n_params;
  const bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(head, 4, 4, f) == 4 &&
                  std::fwrite(&np, 8, 1, f) == 1 &&
                  std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  return (std::fclose(f) == 0 && ok) ? 0 : MGRHD_E_OPTION;
}

int mgrhd_mlp_load(mgrhd_mlp* m, const char* path) {
  if (!m || !path) return MGRHD_E_NULL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return MGRHD_E_OPTION;
  char magic[8];
  int32_t head[4];
  int64_t np = -1;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
            std::fread(head, 4, 4, f) == 4 && std::fread(&np, 8, 1, f) == 1;
  // the file must describe this network exactly
  ok = ok && head[0] == 1 && head[1] == m->n_in && head[2] == m->n_hidden &&
       head[3] == m->n_out && np == m->n_params;
  std::vector<float> p(ok ? (size_t)np : 0);
  ok = ok && std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  if (!ok) return MGRHD_E_SIZE;
  return mgrhd_mlp_set_params(m, p.data());
}

int mgrhd_mlp_forward(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows, float* Y,
                      mgrhd_stream_t stream) {
  if (!m || !X_fm || !Y) return MGRHD_E_NULL;
  if (rows < 0 || ld_x < rows) return MGRHD_E_SIZE;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t r0 = 0; r0 < rows; r0 += m->max_rows) {
    const int64_t r = std::min(m->max_rows, rows - r0);
    forward(m, s, X_fm + r0, ld_x, r, Y + r0 * m->n_out, false);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_gradients(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows,
                        const float* Y_target, float* loss_out, mgrhd_stream_t stream) {
  if (!m || !X_fm || !Y_target) return MGRHD_E_NULL;
  if (rows < 1 || rows > m->max_rows || ld_x < rows) return MGRHD_E_SIZE;
  hipStream_t s = (hipStream_t)stream;
  forward(m, s, X_fm, ld_x, rows, m->Y, true);
  backward(m, s, X_fm, ld_x, rows, Y_target);
  if (loss_out)
    (void)hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_adam_step(mgrhd_mlp* m, float lr, mgrhd_stream_t stream) {
  if (!m) return MGRHD_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  m->step += 1;
  m->dirty = true;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, grid1(m->n_params), dim3(256), 0, s, m->params, m->grads, m->adam_m,
                     m->adam_v, m->n_params, lr, b1, b2, 1e-8f, c1, c2);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_train_step(mgrhd_mlp* m, const float* X_fm, int64_t ld_x, int64_t rows,
                         const float* Y_target, float lr, float* loss_out, mgrhd_stream_t stream) {
  int rc = mgrhd_mlp_gradients(m, X_fm, ld_x, rows, Y_target, loss_out, stream);
  if (rc) return rc;
  return mgrhd_mlp_adam_step(m, lr, stream);
}

static int phys_args(PhysArgs& p, const double* E, const double* F, const double* rho,
                     const double* egas, const double* v, int64_t n, const double* edges,
                     const mgrhd_opacity_params* op, double dt, double c_hat,
                     const mgrhd_options* opt) {
  if (!E || !F || !rho || !egas || !v || !edges || !op || !op->chi_lo) return MGRHD_E_NULL;
  if (n < 0 || op->n_groups < 1 || op->n_groups > MGRHD_MAX_GROUPS) return MGRHD_E_SIZE;
  mgrhd_options d;
  mgrhd_default_options(&d);
  if (!opt) opt = &d;
  std::memset(&p, 0, sizeof(p));
  p.E = E;
  p.F = F;
  p.rho = rho;
  p.egas = egas;
  p.v = v;
  p.kappa = op->kappa_scale;
  p.edges = edges;
  p.chi_lo = op->chi_lo;
  p.alpha = op->alpha_chi;
  p.n = n;
  p.ng = op->n_groups;
  p.dt = dt;
  p.chat = c_hat;
  p.c = opt->c;
  p.a = opt->a_rad;
  p.cv = opt->c_v;
  return 0;
}

// Pack the weights for the fused path if they changed, and fill the
// weight, statistic and kind fields of q.  The inference kernels' dynamic LDS
// limit is raised once per process.
static int prepare_infer(mgrhd_mlp* m, hipStream_t s, const float* x_mean, const float* x_istd,
                         const float* y_mean, const float* y_std, int32_t kind, InferArgs& q) {
  static std::once_flag once;
  static bool lds_ok = false;
  std::call_once(once, [] {
    lds_ok = hipFuncSetAttribute((const void*)k_infer, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 96 * 1024) == hipSuccess &&
             hipFuncSetAttribute((const void*)k_infer_items,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 96 * 1024) == hipSuccess;
  });
  if (!lds_ok) return MGRHD_E_DEVICE;
  if (m->dirty) {
    for (int l = 0; l < 4; ++l)
      hipLaunchKernelGGL(k_pack, grid1((int64_t)m->n_pad[l] * m->k_pad[l]), dim3(256), 0, s,
                         m->params + m->w_off[l], m->params + m->b_off[l], m->out_dim[l],
                         m->in_dim[l], m->n_pad[l], m->k_pad[l], m->wpack + m->wp_off[l],
                         m->bpack + m->bp_off[l]);
    m->dirty = false;
  }
  std::memset(&q, 0, sizeof(q));
  q.xmean = x_mean;
  q.xistd = x_istd;
  q.ymean = y_mean;
  q.ystd = y_std;
  for (int l = 0; l < 4; ++l) {
    q.W[l] = m->wpack + m->wp_off[l];
    q.b[l] = m->bpack + m->bp_off[l];
    q.K_pad[l] = m->k_pad[l];
    q.N_pad[l] = m->n_pad[l];
  }
  q.n_in = m->n_in;
  q.n_out = m->n_out;
  q.kind = kind;
  return 0;
}

static int num_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

}  // extern "C"

namespace mgrhd {

int mlp_check_patches(const mgrhd_mlp* m, int32_t n_groups) {
  if (!m) return MGRHD_E_NULL;
  if (m->n_hidden != kHidden || m->n_in != 2 + 3 * n_groups || m->n_out != 1 + n_groups ||
      m->k_pad[0] > kMaxKin)
    return MGRHD_E_SIZE;
  return 0;
}

int mlp_infer_items(mgrhd_mlp* m, const KArgs* d_patches, const BatchItem* d_items, int64_t lo,
                    int64_t hi, int32_t n_groups, int32_t kind, const float* x_mean,
                    const float* x_istd, const float* y_mean, const float* y_std, hipStream_t s) {
  int rc = mlp_check_patches(m, n_groups);
  if (rc) return rc;
  if (!x_mean || !x_istd || !y_mean || !y_std) return MGRHD_E_NULL;
  if (kind < 0 || kind > 1) return MGRHD_E_OPTION;
  if (hi <= lo) return 0;
  InferItemsArgs a;
  if ((rc = prepare_infer(m, s, x_mean, x_istd, y_mean, y_std, kind, a.q)) != 0) return rc;
  a.patches = d_patches;
  a.items = d_items;
  a.lo = lo;
  a.hi = hi;
  const int64_t cap = (int64_t)num_cus() * 4;
  const int64_t blocks = (hi - lo) < cap ? (hi - lo) : cap;
  hipLaunchKernelGGL(k_infer_items, dim3((unsigned)blocks), dim3(256),
                     infer_lds_bytes(m->k_pad[0], n_groups), s, a);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace mgrhd

extern "C" {

int mgrhd_mlp_features(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                       const double* v, int64_t n, const double* group_edges,
                       const mgrhd_opacity_params* op, double dt, double c_hat,
                       const mgrhd_options* opt, const float* mean, const float* inv_std,
                       float* X_fm, mgrhd_stream_t stream) {
  PhysArgs p;
  int rc = phys_args(p, E_g, F_g, rho, e_gas, v, n, group_edges, op, dt, c_hat, opt);
  if (rc) return rc;
  if (!mean || !inv_std || !X_fm) return MGRHD_E_NULL;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_features, grid1(n), dim3(256), 0, (hipStream_t)stream, p, mean, inv_std,
                     X_fm);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_targets(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                      const double* v, int64_t n, const double* group_edges,
                      const mgrhd_opacity_params* op, double dt, double c_hat,
                      const mgrhd_options* opt, const double* E_new, const double* e_gas_new,
                      const double* v_new, float* Y, mgrhd_stream_t stream) {
  PhysArgs p;
  int rc = phys_args(p, E_g, F_g, rho, e_gas, v, n, group_edges, op, dt, c_hat, opt);
  if (rc) return rc;
  if (!E_new || !e_gas_new || !v_new || !Y) return MGRHD_E_NULL;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_targets, grid1(n), dim3(256), 0, (hipStream_t)stream, p, E_new, e_gas_new,
                     v_new, Y);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_guess(const double* E_g, const double* F_g, const double* rho, const double* e_gas,
                    const double* v, int64_t n, const double* group_edges,
                    const mgrhd_opacity_params* op, double dt, double c_hat,
                    const mgrhd_options* opt, const float* Y_norm, const float* y_mean,
                    const float* y_std, int32_t guess_kind, double* guess,
                    mgrhd_stream_t stream) {
  PhysArgs p;
  int rc = phys_args(p, E_g, F_g, rho, e_gas, v, n, group_edges, op, dt, c_hat, opt);
  if (rc) return rc;
  if (!Y_norm || !y_mean || !y_std || !guess) return MGRHD_E_NULL;
  if (guess_kind < 0 || guess_kind > 1) return MGRHD_E_OPTION;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_guess, grid1(n), dim3(256), 0, (hipStream_t)stream, p, Y_norm, y_mean,
                     y_std, opt ? opt->S_g : nullptr, (int)guess_kind, guess);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_infer(mgrhd_mlp* m, const double* E_g, const double* F_g, const double* rho,
                    const double* e_gas, const double* v, int64_t n, const double* group_edges,
                    const mgrhd_opacity_params* op, double dt, double c_hat,
                    const mgrhd_options* opt, const float* x_mean, const float* x_istd,
                    const float* y_mean, const float* y_std, int32_t guess_kind, double* guess,
                    mgrhd_stream_t stream) {
  if (!m) return MGRHD_E_NULL;
  PhysArgs p;
  int rc = phys_args(p, E_g, F_g, rho, e_gas, v, n, group_edges, op, dt, c_hat, opt);
  if (rc) return rc;
  if (!x_mean || !x_istd || !y_mean || !y_std || !guess) return MGRHD_E_NULL;
  if (guess_kind < 0 || guess_kind > 1) return MGRHD_E_OPTION;
  if ((rc = mgrhd::mlp_check_patches(m, p.ng)) != 0) return rc;
  if (n == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  InferArgs q;
  if ((rc = prepare_infer(m, s, x_mean, x_istd, y_mean, y_std, guess_kind, q)) != 0) return rc;
  q.p = p;
  q.S = opt ? opt->S_g : nullptr;
  q.guess = guess;
  const int64_t tiles = (n + kTile - 1) / kTile;
  const int64_t cap = (int64_t)num_cus() * 4;
  const int64_t blocks = tiles < cap ? tiles : cap;
  hipLaunchKernelGGL(k_infer, dim3((unsigned)blocks), dim3(256),
                     infer_lds_bytes(m->k_pad[0], p.ng), s, q);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int mgrhd_mlp_set_fp32_products(mgrhd_mlp* m, int32_t on) {
  if (!m) return MGRHD_E_NULL;
  if (on != 0 && on != 1) return MGRHD_E_OPTION;
  m->fp32 = on != 0;
  return 0;
}

// plain product C = op(A) op(B) through the network's matrix-core kernel
// (BF16 operands, or FP32 operands with fp32 = 1; exposed for tests)
int mgrhd_mlp_gemm(const float* A, int32_t lda, int32_t trans_a, const float* B, int32_t ldb,
                   int32_t trans_b, float* C, int32_t ldc, int64_t M, int32_t N, int32_t K,
                   int32_t fp32, mgrhd_stream_t stream) {
  if (!A || !B || !C) return MGRHD_E_NULL;
  if (M < 0 || N < 0 || K < 0) return MGRHD_E_SIZE;
  if (fp32 != 0 && fp32 != 1) return MGRHD_E_OPTION;
  if (M == 0 || N == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const bool f = fp32 != 0;
  if (trans_a && trans_b)
    gemm<true, true, EPI_NONE>(s, A, lda, B, ldb, nullptr, C, ldc, nullptr, M, N, K, 1, f);
  else if (trans_a)
    gemm<true, false, EPI_NONE>(s, A, lda, B, ldb, nullptr, C, ldc, nullptr, M, N, K, 1, f);
  else if (trans_b)
    gemm<false, true, EPI_NONE>(s, A, lda, B, ldb, nullptr, C, ldc, nullptr, M, N, K, 1, f);
  else
    gemm<false, false, EPI_NONE>(s, A, lda, B, ldb, nullptr, C, ldc, nullptr, M, N, K, 1, f);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

void mgrhd_mlp_destroy(mgrhd_mlp* m) {
  if (!m) return;
  if (m->params) (void)hipFree(m->params);
  if (m->grads) (void)hipFree(m->grads);
  if (m->adam_m) (void)hipFree(m->adam_m);
  if (m->adam_v) (void)hipFree(m->adam_v);
  if (m->act) (void)hipFree(m->act);
  if (m->loss) (void)hipFree(m->loss);
  if (m->wpack) (void)hipFree(m->wpack);
  if (m->bpack) (void)hipFree(m->bpack);
  delete m;
}

}  // extern "C"
