// rtcdf_mlp.hip -- the learned configuration picker: sketch features of an
// input array, a small FP32 MLP (34 -> 64 -> 64 -> 54, ReLU) that predicts the
// (normalised) log runtime of every kernel configuration, its training
// (forward, backward, Adam) and the masked argmin pick.
//
// Parameter layout (one flat float array of kMlpParams entries):
//   W1[64][34] b1[64] W2[64][64] b2[64] W3[54][64] b3[54]
// Training is deterministic: per-sample deltas are stored, and every weight
// gradient is a fixed-order sum over the samples by one thread.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

constexpr int D0 = kMlpIn, H = kMlpHidden, D3 = kMlpOut;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * D0, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + D3 * H, NPARAM = OFF_B3 + D3;
static_assert(NPARAM == kMlpParams, "parameter layout");
static_assert(D3 <= 64 && H == 64, "one 64-thread workgroup computes every unit of a layer");
static_assert(NPARAM * 4 + 1024 < 65536, "the pick kernel stages every weight in LDS");

// ---------------------------------------------------------------- sketch

// Features of one array: [log2 n, log2 R, fraction of the S sample keys in
// each of 32 equal-width bins of the range], S = min(samples, n), sample i at
// position floor(i * n / S).  One workgroup of 256 threads.
__device__ void sketch_block(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R,
                             uint32_t samples, float* feat /* LDS or global, 34 floats */,
                             uint32_t* bins /* LDS, 32 words */) {
  const uint32_t tid = threadIdx.x;
  if (tid < kSketchBins) bins[tid] = 0;
  __syncthreads();
  const uint64_t S = n < samples ? n : samples;
  // The sample loads of a thread are issued together (kBatch in flight), then
  // binned: a scattered load costs a memory latency, not a bandwidth.
  constexpr uint32_t kBatch = 16;
  for (uint64_t i0 = 0; i0 < S; i0 += (uint64_t)kBatch * blockDim.x) {
    int32_t key[kBatch];
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint64_t i = i0 + (uint64_t)k * blockDim.x + tid;
      key[k] = i < S ? keys[(i * n) / S] : 0;
    }
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint64_t i = i0 + (uint64_t)k * blockDim.x + tid;
      if (i < S) {
        const uint64_t b = ((uint64_t)((int64_t)key[k] - minVal) * kSketchBins) / R;
        atomicAdd(&bins[b < kSketchBins ? b : kSketchBins - 1], 1u);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    feat[0] = n ? log2f((float)n) : 0.f;
    feat[1] = log2f((float)R);
  }
  if (tid < kSketchBins) feat[2 + tid] = S ? (float)bins[tid] / (float)S : 0.f;
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_sketch(const int32_t* keys, uint64_t n, int64_t minVal,
                                                uint64_t R, uint32_t samples, float* feat) {
  __shared__ uint32_t bins[kSketchBins];
  __shared__ float f[D0];
  sketch_block(keys, n, minVal, R, samples, f, bins);
  if (threadIdx.x < D0) feat[threadIdx.x] = f[threadIdx.x];
}

// ---------------------------------------------------------------- forward

// One workgroup of 64 threads per sample; thread j computes hidden unit j (and
// output unit j when j < D3 <= 64).  Stores Z1, Z2 (pre-activations) and Y.
__device__ void mlp_forward_sample(const float* P, const float* x, float* z1, float* z2, float* y,
                                   float* h /* LDS, 2 * 64 */) {
  const int j = threadIdx.x;
  float a = P[OFF_B1 + j];
  for (int i = 0; i < D0; ++i) a = fmaf(P[OFF_W1 + j * D0 + i], x[i], a);
  if (z1) z1[j] = a;
  h[j] = fmaxf(a, 0.f);
  __syncthreads();
  float b = P[OFF_B2 + j];
  for (int i = 0; i < H; ++i) b = fmaf(P[OFF_W2 + j * H + i], h[i], b);
  if (z2) z2[j] = b;
  h[H + j] = fmaxf(b, 0.f);
  __syncthreads();
  if (j < D3) {
    float c = P[OFF_B3 + j];
    for (int i = 0; i < H; ++i) c = fmaf(P[OFF_W3 + j * H + i], h[H + i], c);
    y[j] = c;
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_mlp_forward(const float* P, const float* X, uint32_t B, float* Z1,
                                                    float* Z2, float* Y) {
  __shared__ float h[2 * H];
  __shared__ float x[D0];
  const uint32_t s = blockIdx.x;
  if (s >= B) return;
  if (threadIdx.x < D0) x[threadIdx.x] = X[(size_t)s * D0 + threadIdx.x];
  __syncthreads();
  mlp_forward_sample(P, x, Z1 ? Z1 + (size_t)s * H : nullptr, Z2 ? Z2 + (size_t)s * H : nullptr,
                     Y + (size_t)s * D3, h);
}

// ---------------------------------------------------------------- backward

// Per-sample deltas of the masked mean squared error
// L = sum(M (Y - T)^2) / count: dY = 2 M (Y - T) / count, dZ2 = (W3^T dY) [Z2 > 0],
// dZ1 = (W2^T dZ2) [Z1 > 0].  Also the per-sample loss terms.
__global__ __launch_bounds__(64) void k_mlp_deltas(const float* P, const float* Z1, const float* Z2,
                                                   const float* Y, const float* T, const float* M,
                                                   uint32_t B, float inv_count, float* dY, float* dZ1,
                                                   float* dZ2, float* lossterm) {
  __shared__ float dy[D3];
  __shared__ float dz2[H];
  __shared__ float lt[64];
  const uint32_t s = blockIdx.x;
  const int j = threadIdx.x;
  if (s >= B) return;
  float l = 0.f;
  if (j < D3) {
    const size_t o = (size_t)s * D3 + j;
    const float e = Y[o] - T[o];
    const float d = 2.f * M[o] * e * inv_count;
    dy[j] = d;
    dY[o] = d;
    l = M[o] * e * e;
  }
  lt[j] = l;
  __syncthreads();
  float g = 0.f;
  for (int k = 0; k < D3; ++k) g = fmaf(P[OFF_W3 + k * H + j], dy[k], g);
  g = Z2[(size_t)s * H + j] > 0.f ? g : 0.f;
  dz2[j] = g;
  dZ2[(size_t)s * H + j] = g;
  __syncthreads();
  float g1 = 0.f;
  for (int k = 0; k < H; ++k) g1 = fmaf(P[OFF_W2 + k * H + j], dz2[k], g1);
  dZ1[(size_t)s * H + j] = Z1[(size_t)s * H + j] > 0.f ? g1 : 0.f;
  if (j == 0) {
    float acc = 0.f;
    for (int k = 0; k < 64; ++k) acc += lt[k];
    lossterm[s] = acc;
  }
}

// Weight and bias gradients: one thread per parameter, summing over the
// samples in index order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* X, const float* Z1, const float* Z2,
                                                   const float* dY, const float* dZ1, const float* dZ2,
                                                   uint32_t B, float* G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float* delta;
  const float* act = nullptr;     // nullptr: bias (activation 1)
  int dstride, astride, j, i = 0;
  bool relu_act = false;
  if (p < OFF_B1) {
    j = (p - OFF_W1) / D0; i = (p - OFF_W1) % D0; delta = dZ1; dstride = H; act = X; astride = D0;
  } else if (p < OFF_W2) {
    j = p - OFF_B1; delta = dZ1; dstride = H; astride = 0;
  } else if (p < OFF_B2) {
    j = (p - OFF_W2) / H; i = (p - OFF_W2) % H; delta = dZ2; dstride = H; act = Z1; astride = H;
    relu_act = true;
  } else if (p < OFF_W3) {
    j = p - OFF_B2; delta = dZ2; dstride = H; astride = 0;
  } else if (p < OFF_B3) {
    j = (p - OFF_W3) / H; i = (p - OFF_W3) % H; delta = dY; dstride = D3; act = Z2; astride = H;
    relu_act = true;
  } else {
    j = p - OFF_B3; delta = dY; dstride = D3; astride = 0;
  }
  float g = 0.f;
  for (uint32_t s = 0; s < B; ++s) {
    float a = 1.f;
    if (act) {
      a = act[(size_t)s * astride + i];
      if (relu_act) a = fmaxf(a, 0.f);
    }
    g = fmaf(delta[(size_t)s * dstride + j], a, g);
  }
  G[p] = g;
}

// One Adam step (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
// The coefficients 1 - b1 and 1 - b2 come from the host in double precision
// (1.f - 0.999f is 1.3e-5 off in float).
__global__ __launch_bounds__(256) void k_adam(float* P, const float* G, float* Mo, float* Vo, float lr,
                                              float b1, float b2, float omb1, float omb2, float eps,
                                              float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = G[p];
  const float m = b1 * Mo[p] + omb1 * g;
  const float v = b2 * Vo[p] + omb2 * g * g;
  Mo[p] = m;
  Vo[p] = v;
  P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void k_sum_loss(const float* lossterm, uint32_t B, float inv_count, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (uint32_t i = 0; i < B; ++i) s += lossterm[i];
    out[0] = s * inv_count;
  }
}

// ---------------------------------------------------------------- pick

// The network and the masked argmin for one array, by one workgroup of 256
// threads, from the raw features f (LDS, D0 floats; standardised in place).
// The weights are first staged into LDS (Ps) with coalesced loads; each unit's
// dot product is split over 4 threads and combined with lane shuffles.
__device__ void pick_block(const float* P, const float* norm, const uint8_t* valid, float* f, float* Ps,
                           float* h, float* y, uint32_t* out_index, float* out_pred, float* out_zmax,
                           float* out_feat) {
  {
    // every load of the staging is issued before the first store (16-byte
    // vectors; P and Ps are 16-byte aligned), then the scalar tail
    typedef float v4f __attribute__((ext_vector_type(4)));
    constexpr int kV = NPARAM / 4, kPer = (kV + 255) / 256;
    const v4f* P4 = reinterpret_cast<const v4f*>(P);
    v4f r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * 256;
      r[k] = P4[i < kV ? i : kV - 1];
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * 256;
      if (i < kV) reinterpret_cast<v4f*>(Ps)[i] = r[k];
    }
    for (int i = 4 * kV + (int)threadIdx.x; i < NPARAM; i += 256) Ps[i] = P[i];
  }
  if (out_feat && threadIdx.x < D0) out_feat[threadIdx.x] = f[threadIdx.x];
  __syncthreads();
  if (threadIdx.x < D0) f[threadIdx.x] = (f[threadIdx.x] - norm[threadIdx.x]) / norm[D0 + threadIdx.x];
  __syncthreads();
  if (out_zmax && threadIdx.x == 0) {   // distance from the training features, in sd units
    float z = 0.f;
    for (int i = 0; i < D0; ++i) z = fmaxf(z, fabsf(f[i]));
    out_zmax[0] = z;
  }
  // unit j of a layer: threads 4j .. 4j + 3, thread q sums the inputs i = q mod 4
  const int j = threadIdx.x >> 2, q = threadIdx.x & 3;
  float a = 0.f;
  for (int i = q; i < D0; i += 4) a = fmaf(Ps[OFF_W1 + j * D0 + i], f[i], a);
  a += __shfl_xor(a, 1, 64);
  a += __shfl_xor(a, 2, 64);
  if (q == 0) h[j] = fmaxf(a + Ps[OFF_B1 + j], 0.f);
  __syncthreads();
  float b = 0.f;
  for (int i = q; i < H; i += 4) b = fmaf(Ps[OFF_W2 + j * H + i], h[i], b);
  b += __shfl_xor(b, 1, 64);
  b += __shfl_xor(b, 2, 64);
  if (q == 0) h[H + j] = fmaxf(b + Ps[OFF_B2 + j], 0.f);
  __syncthreads();
  float c = 0.f;
  if (j < D3)
    for (int i = q; i < H; i += 4) c = fmaf(Ps[OFF_W3 + j * H + i], h[H + i], c);
  c += __shfl_xor(c, 1, 64);
  c += __shfl_xor(c, 2, 64);
  if (j < D3 && q == 0) {
    c += Ps[OFF_B3 + j];
    y[j] = c;
    if (out_pred) out_pred[j] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = -1;
    for (int k = 0; k < D3; ++k)
      if (valid[k] && (best < 0 || y[k] < y[best])) best = k;
    out_index[0] = (uint32_t)best;
  }
}

// Sketch -> standardised features -> MLP -> argmin over the valid
// configurations (lowest index on ties).  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_pick(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R,
                                              uint32_t samples, const float* P, const float* norm,
                                              const uint8_t* valid, uint32_t* out_index, float* out_pred,
                                              float* out_zmax, float* out_feat) {
  __shared__ __align__(16) float Ps[NPARAM];
  __shared__ uint32_t bins[kSketchBins];
  __shared__ float f[D0];
  __shared__ float h[2 * H];
  __shared__ float y[D3];
  sketch_block(keys, n, minVal, R, samples, f, bins);
  pick_block(P, norm, valid, f, Ps, h, y, out_index, out_pred, out_zmax, out_feat);
}

// The same pick with the sampling spread over gridDim.x workgroups (the
// sample loads are scattered over the whole array, and one compute unit keeps
// only so many misses in flight).  Each workgroup bins its share of the S
// samples (sample i at position floor(i n / S), as in sketch_block) and adds
// its bin counts to acc[0, 32); the last workgroup to finish (counter
// acc[32]) reads them, returns acc to zero for the next pick and runs the
// network.  acc must be zero on entry.
__global__ __launch_bounds__(256) void k_pick_spread(const int32_t* keys, uint64_t n, int64_t minVal,
                                                     uint64_t R, uint32_t samples, const float* P,
                                                     const float* norm, const uint8_t* valid,
                                                     uint32_t* acc, uint32_t* out_index, float* out_pred,
                                                     float* out_zmax, float* out_feat) {
  __shared__ __align__(16) float Ps[NPARAM];
  __shared__ uint32_t bins[kSketchBins];
  __shared__ float f[D0];
  __shared__ float h[2 * H];
  __shared__ float y[D3];
  __shared__ uint32_t last;
  const uint32_t tid = threadIdx.x, G = gridDim.x, w = blockIdx.x;
  if (tid < kSketchBins) bins[tid] = 0;
  __syncthreads();
  const uint64_t S = n < samples ? n : samples;
  const uint64_t i0 = S * w / G, i1 = S * (w + 1) / G;
  constexpr uint32_t kBatch = 4;
  for (uint64_t b0 = i0; b0 < i1; b0 += (uint64_t)kBatch * 256) {
    int32_t key[kBatch];
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint64_t i = b0 + (uint64_t)k * 256 + tid;
      key[k] = i < i1 ? keys[(i * n) / S] : 0;
    }
#pragma unroll
    for (uint32_t k = 0; k < kBatch; ++k) {
      const uint64_t i = b0 + (uint64_t)k * 256 + tid;
      if (i < i1) {
        const uint64_t b = ((uint64_t)((int64_t)key[k] - minVal) * kSketchBins) / R;
        atomicAdd(&bins[b < kSketchBins ? b : kSketchBins - 1], 1u);
      }
    }
  }
  __syncthreads();
  if (tid < kSketchBins && bins[tid]) atomicAdd(&acc[tid], bins[tid]);
  __threadfence();   // this workgroup's counts are visible before it is counted as done
  __syncthreads();
  if (tid == 0) last = atomicAdd(&acc[kSketchBins], 1u) == G - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (tid < kSketchBins) {
    const uint32_t c = __hip_atomic_load(&acc[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    f[2 + tid] = S ? (float)c / (float)S : 0.f;
    acc[tid] = 0u;
  }
  if (tid == 0) {
    acc[kSketchBins] = 0u;
    f[0] = n ? log2f((float)n) : 0.f;
    f[1] = log2f((float)R);
  }
  __syncthreads();
  pick_block(P, norm, valid, f, Ps, h, y, out_index, out_pred, out_zmax, out_feat);
}

}  // namespace

hipError_t launch_sketch(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R, uint32_t samples,
                         float* feat, hipStream_t s) {
  hipLaunchKernelGGL(k_sketch, dim3(1), dim3(256), 0, s, keys, n, minVal, R, samples, feat);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, uint32_t B, float* Z1, float* Z2, float* Y,
                              hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(64), 0, s, P, X, B, Z1, Z2, Y);
  return hipGetLastError();
}

// Gradient of the masked MSE at P over the batch (X, T, M) into G; loss into
// *loss_dev.  scratch: 4 * B * H + 2 * B * D3 + B floats.
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const float* M, uint32_t B,
                           float inv_count, float* G, float* loss_dev, float* scratch, hipStream_t s) {
  if (B == 0) return hipSuccess;
  float* Z1 = scratch;
  float* Z2 = Z1 + (size_t)B * H;
  float* Y = Z2 + (size_t)B * H;
  float* dY = Y + (size_t)B * D3;
  float* dZ1 = dY + (size_t)B * D3;
  float* dZ2 = dZ1 + (size_t)B * H;
  float* lt = dZ2 + (size_t)B * H;
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(64), 0, s, P, X, B, Z1, Z2, Y);
  hipLaunchKernelGGL(k_mlp_deltas, dim3(B), dim3(64), 0, s, P, Z1, Z2, Y, T, M, B, inv_count, dY, dZ1,
                     dZ2, lt);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((NPARAM + 255) / 256), dim3(256), 0, s, X, Z1, Z2, dY, dZ1, dZ2, B,
                     G);
  if (loss_dev) hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, s, lt, B, inv_count, loss_dev);
  return hipGetLastError();
}

size_t mlp_grad_scratch_floats(uint32_t B) { return (size_t)B * (4 * H + 2 * D3 + 1); }

hipError_t launch_adam(float* P, const float* G, float* Mo, float* Vo, float lr, float b1, float b2,
                       float eps, uint32_t t, hipStream_t s) {
  const double db1 = b1, db2 = b2;
  const float c1 = (float)(1.0 - std::pow(db1, (double)t)), c2 = (float)(1.0 - std::pow(db2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, G, Mo, Vo, lr, b1, b2,
                     (float)(1.0 - db1), (float)(1.0 - db2), eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pick(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R, uint32_t samples,
                       const float* P, const float* norm, const uint8_t* valid, uint32_t* out_index,
                       float* out_pred, float* out_zmax, float* out_feat, hipStream_t s, uint32_t* acc) {
  if (acc != nullptr) {
    hipLaunchKernelGGL(k_pick_spread, dim3(kPickGroups), dim3(256), 0, s, keys, n, minVal, R, samples, P, norm,
                       valid, acc, out_index, out_pred, out_zmax, out_feat);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_pick, dim3(1), dim3(256), 0, s, keys, n, minVal, R, samples, P, norm, valid,
                     out_index, out_pred, out_zmax, out_feat);
  return hipGetLastError();
}

}  // namespace rtcdf
