// sample_p3p.hip -- minimal sampling (Philox4x64-10) and float64 P3P, one
// lane per sample, candidates compacted per workgroup (ImLoc Sec. 3.3, "Pose
// Estimation": batches of minimal sets, P3P hypotheses).
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kP3PBlock = 256;

__global__ __launch_bounds__(kP3PBlock) void sample_p3p_kernel(
    const float* __restrict__ U, const float* __restrict__ V, const float* __restrict__ X,
    const float* __restrict__ Y, const float* __restrict__ Z, int64_t m, Cam K, uint64_t seed, uint64_t query,
    int exhaustive, int64_t h0, int64_t count, double inv_tau, double* __restrict__ out_pose, float* __restrict__ out_proj,
    int64_t* __restrict__ out_h, int32_t* __restrict__ out_j, int32_t* __restrict__ n_cand,
    int32_t* __restrict__ triples) {
  const int64_t s = (int64_t)blockIdx.x * kP3PBlock + threadIdx.x;
  Pose sol[4];
  int ns = 0;
  if (s < count) {
    const uint64_t h = (uint64_t)(h0 + s);
    int idx[3] = {-1, -1, -1};
    const bool ok = exhaustive ? unrank_triple(h, (uint64_t)m, idx) : sample_triple(seed, query, h, (uint64_t)m, idx);
    if (triples) {
      triples[3 * s] = ok ? idx[0] : -1;
      triples[3 * s + 1] = ok ? idx[1] : -1;
      triples[3 * s + 2] = ok ? idx[2] : -1;
    }
    if (ok) {
      double y[3][3], x[3][3];
      for (int k = 0; k < 3; ++k) {
        const int i = idx[k];
        const double bx = ((double)U[i] - K.cx) / K.fx, by = ((double)V[i] - K.cy) / K.fy;
        const double inv = 1.0 / sqrt(bx * bx + by * by + 1.0);
        y[k][0] = bx * inv; y[k][1] = by * inv; y[k][2] = inv;
        x[k][0] = X[i]; x[k][1] = Y[i]; x[k][2] = Z[i];
      }
      ns = p3p_pencil(y, x, sol);
    }
  }
  // workgroup-wide exclusive scan of the solution counts (keeps sample order
  // inside the workgroup; workgroups append in completion order)
  __shared__ int s_scan[kP3PBlock];
  __shared__ int s_base;
  s_scan[threadIdx.x] = ns;
  __syncthreads();
  for (int off = 1; off < kP3PBlock; off <<= 1) {
    const int v = threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0;
    __syncthreads();
    s_scan[threadIdx.x] += v;
    __syncthreads();
  }
  if (threadIdx.x == kP3PBlock - 1) s_base = s_scan[kP3PBlock - 1] > 0 ? atomicAdd(n_cand, s_scan[kP3PBlock - 1]) : 0;
  __syncthreads();
  const int base = s_base + s_scan[threadIdx.x] - ns;
  for (int j = 0; j < ns; ++j) {
    const int64_t o = base + j;
    for (int e = 0; e < 9; ++e) out_pose[12 * o + e] = sol[j].R[e];
    for (int e = 0; e < 3; ++e) out_pose[12 * o + 9 + e] = sol[j].t[e];
    double M[12];
    projection_rows(sol[j], K, M);
    float4* pr = reinterpret_cast<float4*>(out_proj + 16 * o);
    pr[0] = make_float4((float)(M[0] * inv_tau), (float)(M[1] * inv_tau), (float)(M[2] * inv_tau), (float)(M[3] * inv_tau));
    pr[1] = make_float4((float)(M[4] * inv_tau), (float)(M[5] * inv_tau), (float)(M[6] * inv_tau), (float)(M[7] * inv_tau));
    pr[2] = make_float4((float)M[8], (float)M[9], (float)M[10], (float)M[11]);
    pr[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    out_h[o] = h0 + s;
    out_j[o] = j;
  }
}

hipError_t launch_sample_p3p(const CorrF32& c, int64_t m, CamH K, uint64_t seed, uint64_t query, int exhaustive,
                             int64_t h0, int64_t count, double tau, const CandBuf& cb, int32_t* triples, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)((count + kP3PBlock - 1) / kP3PBlock);
  Cam k{K.fx, K.fy, K.cx, K.cy};
  hipLaunchKernelGGL(sample_p3p_kernel, dim3(blocks), dim3(kP3PBlock), 0, s, c.u, c.v, c.X, c.Y, c.Z, m, k, seed,
                     query, exhaustive, h0, count, 1.0 / tau, cb.pose, cb.proj, cb.h, cb.j, cb.n, triples);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Float32 projection rows of the scoring kernel: rows a and b divided by tau.
__global__ void make_proj_kernel(const double* __restrict__ poses, int64_t np, Cam K, double inv_tau,
                                 float* __restrict__ proj) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  Pose P;
  for (int e = 0; e < 9; ++e) P.R[e] = poses[12 * i + e];
  for (int e = 0; e < 3; ++e) P.t[e] = poses[12 * i + 9 + e];
  double M[12];
  projection_rows(P, K, M);
  for (int e = 0; e < 12; ++e) proj[16 * i + e] = (float)(e < 8 ? M[e] * inv_tau : M[e]);
  for (int e = 12; e < 16; ++e) proj[16 * i + e] = 0.f;
}

hipError_t launch_make_proj(const double* poses, int64_t np, CamH K, double tau, float* proj, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  Cam k{K.fx, K.fy, K.cx, K.cy};
  hipLaunchKernelGGL(make_proj_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, poses, np, k, 1.0 / tau,
                     proj);
  return hipGetLastError();
}

// Scoring-set gather: S_j = point floor(j * n / m), j < m.
__global__ void gather_subset_kernel(const float* __restrict__ U, const float* __restrict__ V,
                                     const float* __restrict__ X, const float* __restrict__ Y,
                                     const float* __restrict__ Z, const float* __restrict__ W, int64_t n, int64_t m,
                                     float* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = (int64_t)(((uint64_t)j * (uint64_t)n) / (uint64_t)m);  // n < 2^31: no overflow
  dst[j] = U[i];
  dst[m + j] = V[i];
  dst[2 * m + j] = X[i];
  dst[3 * m + j] = Y[i];
  dst[4 * m + j] = Z[i];
  dst[5 * m + j] = W ? W[i] : 1.0f;
}

hipError_t launch_gather_subset(const CorrF32& c, int64_t n, int64_t m, float* dst, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_subset_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, c.u, c.v, c.X, c.Y,
                     c.Z, c.w, n, m, dst);
  return hipGetLastError();
}

}  // namespace imloc
