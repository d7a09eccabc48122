// lift.hip -- a world point for every query-to-database match, through the
// stored depth maps (ImLoc Sec. 3.3 "Query Time Matching and 2D-3D Lifting": bilinear depth
// at sub-pixel database coordinates, plain lookup otherwise; keep matches with
// valid depth and confidence above the threshold).
//
// One thread per match.  The output is a stable compaction in match order:
// pass 1 counts the kept matches of every workgroup, pass 2 scans the counts,
// pass 3 recomputes each lift and writes it at its workgroup offset plus its
// rank inside the workgroup.  The arithmetic is float64, rounded once to the
// float32 outputs; the work is a gather of four depth texels per match.
//
// Depth maps come as float32 metres or as 8-bit log-depth codes (Sec. 3.3
// "Data Compression": depth clipped to [0.25, 128] m, quantised uniformly in
// log depth; code 0 = no depth, code c >= 1 = 0.25 * 512^((c - 1) / 254)).
// Code maps are decoded through a 256-entry float64 table each workgroup
// builds in LDS, so a tap costs one byte of HBM instead of four.
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kLiftBlock = 256;

__device__ inline bool depth_ok(float d) { return d > 0.0f && d <= 3.402823466e38f; }  // finite and positive

// Depth texel idx of view map D; false if it holds no valid depth.
template <bool kCodes>
__device__ inline bool tap(const LiftArgs& a, int64_t idx, const double* lut, double& d) {
  if constexpr (kCodes) {
    const int c = a.codes[idx];
    d = lut[c];
    return c != 0;
  } else {
    const float f = a.depth[idx];
    d = f;
    return depth_ok(f);
  }
}

template <bool kCodes>
__device__ inline bool lift_one(const LiftArgs& a, int64_t i, const double* lut, float out[6]) {
  const float conf = a.conf[i];
  if (!(conf > a.min_conf)) return false;
  const int k = a.view[i];
  if (k < 0 || k >= a.n_views) return false;
  const float qu = a.q_u[i], qv = a.q_v[i], fu = a.db_u[i], fv = a.db_v[i];
  if (!isfinite(qu) || !isfinite(qv) || !isfinite(fu) || !isfinite(fv)) return false;
  const int64_t base = (int64_t)k * a.H * a.W;
  const double du = fu, dv = fv;
  double d;
  if (a.subpixel) {
    const double x = du - 0.5, y = dv - 0.5;
    const double x0 = floor(x), y0 = floor(y);
    if (x0 < 0.0 || y0 < 0.0 || x0 + 1.0 > (double)(a.W - 1) || y0 + 1.0 > (double)(a.H - 1)) return false;
    const int64_t c0 = (int64_t)x0, r0 = (int64_t)y0;
    double d00, d01, d10, d11;
    const bool ok00 = tap<kCodes>(a, base + r0 * a.W + c0, lut, d00);
    const bool ok01 = tap<kCodes>(a, base + r0 * a.W + c0 + 1, lut, d01);
    const bool ok10 = tap<kCodes>(a, base + (r0 + 1) * a.W + c0, lut, d10);
    const bool ok11 = tap<kCodes>(a, base + (r0 + 1) * a.W + c0 + 1, lut, d11);
    if (!(ok00 && ok01 && ok10 && ok11)) return false;
    const double ax = x - x0, ay = y - y0;
    d = (1.0 - ay) * ((1.0 - ax) * d00 + ax * d01) + ay * ((1.0 - ax) * d10 + ax * d11);
  } else {
    const double cf = floor(du), rf = floor(dv);
    if (cf < 0.0 || rf < 0.0 || cf > (double)(a.W - 1) || rf > (double)(a.H - 1)) return false;
    if (!tap<kCodes>(a, base + (int64_t)rf * a.W + (int64_t)cf, lut, d)) return false;
  }
  const double* cam = a.cams + 4 * k;
  const double* T = a.poses + 12 * k;
  const double xc = d * (du - cam[2]) / cam[0] - T[9];
  const double yc = d * (dv - cam[3]) / cam[1] - T[10];
  const double zc = d - T[11];
  // X_w = R^T (x_c - t)
  out[0] = qu;
  out[1] = qv;
  out[2] = (float)(T[0] * xc + T[3] * yc + T[6] * zc);
  out[3] = (float)(T[1] * xc + T[4] * yc + T[7] * zc);
  out[4] = (float)(T[2] * xc + T[5] * yc + T[8] * zc);
  out[5] = conf;
  return true;
}

// decode table of the code maps (kLiftBlock == 256: one entry per thread)
template <bool kCodes>
__device__ inline void fill_lut(double* lut) {
  static_assert(kLiftBlock == 256, "one table entry per thread");
  if constexpr (kCodes) {
    lut[threadIdx.x] = log8_level((int)threadIdx.x);
    __syncthreads();
  }
}

template <bool kCodes>
__global__ __launch_bounds__(kLiftBlock) void lift_count_kernel(LiftArgs a) {
  __shared__ double lut[kCodes ? 256 : 1];
  fill_lut<kCodes>(lut);
  const int64_t i = (int64_t)blockIdx.x * kLiftBlock + threadIdx.x;
  float o[6];
  const bool keep = i < a.n && lift_one<kCodes>(a, i, lut, o);
  const int c = __syncthreads_count(keep);
  if (threadIdx.x == 0) a.block_counts[blockIdx.x] = c;
}

// Exclusive scan of the workgroup counts (one workgroup; each thread scans a
// contiguous segment, then the segment totals are scanned).
__global__ __launch_bounds__(1024) void lift_scan_kernel(int32_t* counts, int nb, int32_t* total) {
  __shared__ int s[1024];
  const int seg = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * seg, b1 = min(nb, b0 + seg);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += counts[b];
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  int run = s[threadIdx.x] - sum;
  for (int b = b0; b < b1; ++b) {
    const int c = counts[b];
    counts[b] = run;
    run += c;
  }
  if (threadIdx.x == 1023) *total = s[1023];
}

template <bool kCodes>
__global__ __launch_bounds__(kLiftBlock) void lift_write_kernel(LiftArgs a) {
  __shared__ double lut[kCodes ? 256 : 1];
  fill_lut<kCodes>(lut);
  const int64_t i = (int64_t)blockIdx.x * kLiftBlock + threadIdx.x;
  float o[6];
  const bool keep = i < a.n && lift_one<kCodes>(a, i, lut, o);
  __shared__ int s[kLiftBlock];
  s[threadIdx.x] = keep ? 1 : 0;
  __syncthreads();
  for (int off = 1; off < kLiftBlock; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  if (!keep) return;
  const int64_t dst = (int64_t)a.block_counts[blockIdx.x] + s[threadIdx.x] - 1;
  if (dst >= a.capacity) return;
  a.out_u[dst] = o[0];
  a.out_v[dst] = o[1];
  a.out_X[dst] = o[2];
  a.out_Y[dst] = o[3];
  a.out_Z[dst] = o[4];
  if (a.out_w) a.out_w[dst] = o[5];
  if (a.out_src) a.out_src[dst] = (int32_t)i;
}

int lift_blocks(int64_t n) { return (int)((n + kLiftBlock - 1) / kLiftBlock); }

hipError_t launch_lift(const LiftArgs& a, hipStream_t s) {
  const int nb = lift_blocks(a.n);
  if (nb == 0) return launch_fill_i32(a.n_out, 1, 0, s);
  if (a.codes) {
    hipLaunchKernelGGL(lift_count_kernel<true>, dim3(nb), dim3(kLiftBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(lift_count_kernel<false>, dim3(nb), dim3(kLiftBlock), 0, s, a);
  }
  hipLaunchKernelGGL(lift_scan_kernel, dim3(1), dim3(1024), 0, s, a.block_counts, nb, a.n_out);
  if (a.codes) {
    hipLaunchKernelGGL(lift_write_kernel<true>, dim3(nb), dim3(kLiftBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(lift_write_kernel<false>, dim3(nb), dim3(kLiftBlock), 0, s, a);
  }
  return hipGetLastError();
}

// Encoder of the code maps: nearest level in log depth (halves away from
// zero), depth clipped to [0.25, 128] m, code 0 for depth not finite or <= 0.
// Four depths per thread (one float4 load, one 32-bit store) over the first
// 4 * n4 entries, one per thread over the rest (n4 = 0 when the arrays are
// not 16- and 4-byte aligned).
__global__ __launch_bounds__(256) void log8_encode_kernel(const float* __restrict__ depth, int64_t n, int64_t n4,
                                                           uint8_t* __restrict__ codes) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n4) {
    const float4 v = reinterpret_cast<const float4*>(depth)[q];
    const uint32_t w = (uint32_t)log8_code(v.x) | ((uint32_t)log8_code(v.y) << 8) |
                       ((uint32_t)log8_code(v.z) << 16) | ((uint32_t)log8_code(v.w) << 24);
    reinterpret_cast<uint32_t*>(codes)[q] = w;
  } else {
    const int64_t i = 4 * n4 + (q - n4);
    if (i < n) codes[i] = log8_code(depth[i]);
  }
}

hipError_t launch_log8_encode(const float* depth, int64_t n, uint8_t* codes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool vec = reinterpret_cast<uintptr_t>(depth) % 16 == 0 && reinterpret_cast<uintptr_t>(codes) % 4 == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  const int64_t threads = n4 + (n - 4 * n4);
  hipLaunchKernelGGL(log8_encode_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, depth, n, n4,
                     codes);
  return hipGetLastError();
}

}  // namespace imloc
