// lift.hip -- 2D-2D matches to 2D-3D correspondences through the stored depth
// maps (ImLoc Sec. 3.3 "Query Time Matching and 2D-3D Lifting": bilinear depth
// at sub-pixel database coordinates, plain lookup otherwise; keep matches with
// valid depth and confidence above the threshold).
//
// One thread per match.  The output is a stable compaction in match order:
// pass 1 counts the kept matches of every workgroup, pass 2 scans the counts,
// pass 3 recomputes each lift and writes it at its workgroup offset plus its
// rank inside the workgroup.  The arithmetic is float64, rounded once to the
// float32 outputs; the work is a gather of four depth texels per match.
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kLiftBlock = 256;

__device__ inline bool depth_ok(float d) { return d > 0.0f && d <= 3.402823466e38f; }  // finite and positive

__device__ inline bool lift_one(const LiftArgs& a, int64_t i, float out[6]) {
  const float conf = a.conf[i];
  if (!(conf > a.min_conf)) return false;
  const int k = a.view[i];
  if (k < 0 || k >= a.n_views) return false;
  const float qu = a.q_u[i], qv = a.q_v[i], fu = a.db_u[i], fv = a.db_v[i];
  if (!isfinite(qu) || !isfinite(qv) || !isfinite(fu) || !isfinite(fv)) return false;
  const float* D = a.depth + (int64_t)k * a.H * a.W;
  const double du = fu, dv = fv;
  double d;
  if (a.subpixel) {
    const double x = du - 0.5, y = dv - 0.5;
    const double x0 = floor(x), y0 = floor(y);
    if (x0 < 0.0 || y0 < 0.0 || x0 + 1.0 > (double)(a.W - 1) || y0 + 1.0 > (double)(a.H - 1)) return false;
    const int64_t c0 = (int64_t)x0, r0 = (int64_t)y0;
    const float d00 = D[r0 * a.W + c0], d01 = D[r0 * a.W + c0 + 1];
    const float d10 = D[(r0 + 1) * a.W + c0], d11 = D[(r0 + 1) * a.W + c0 + 1];
    if (!depth_ok(d00) || !depth_ok(d01) || !depth_ok(d10) || !depth_ok(d11)) return false;
    const double ax = x - x0, ay = y - y0;
    d = (1.0 - ay) * ((1.0 - ax) * d00 + ax * d01) + ay * ((1.0 - ax) * d10 + ax * d11);
  } else {
    const double cf = floor(du), rf = floor(dv);
    if (cf < 0.0 || rf < 0.0 || cf > (double)(a.W - 1) || rf > (double)(a.H - 1)) return false;
    const float dd = D[(int64_t)rf * a.W + (int64_t)cf];
    if (!depth_ok(dd)) return false;
    d = dd;
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

__global__ __launch_bounds__(kLiftBlock) void lift_count_kernel(LiftArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kLiftBlock + threadIdx.x;
  float o[6];
  const bool keep = i < a.n && lift_one(a, i, o);
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

__global__ __launch_bounds__(kLiftBlock) void lift_write_kernel(LiftArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kLiftBlock + threadIdx.x;
  float o[6];
  const bool keep = i < a.n && lift_one(a, i, o);
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
  hipLaunchKernelGGL(lift_count_kernel, dim3(nb), dim3(kLiftBlock), 0, s, a);
  hipLaunchKernelGGL(lift_scan_kernel, dim3(1), dim3(1024), 0, s, a.block_counts, nb, a.n_out);
  hipLaunchKernelGGL(lift_write_kernel, dim3(nb), dim3(kLiftBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace imloc
