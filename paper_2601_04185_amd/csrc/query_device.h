// query_device.h -- device helpers over a query descriptor: the camera a
// candidate pose is seen through (one camera, or a rig camera composed with
// the rig pose) and the float32 projection rows of a candidate slot.
#pragma once

#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

// The pose of candidate P seen by camera `cam` of the query: for a rig,
// cam_from_world = (R_c R, R_c t + t_c) with the camera's intrinsics.
__device__ inline void camera_pose(const QueryDesc& d, int cam, const Pose& P, Pose& Pc, Cam& K) {
  if (d.ncam == 0) {
    Pc = P;
    K = Cam{d.fx, d.fy, d.cx, d.cy};
    return;
  }
  const double* rc = d.rig + 16 * cam;
  K = Cam{rc[0], rc[1], rc[2], rc[3]};
  const double* Rc = rc + 4;
  const double* tc = rc + 13;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Pc.R[3 * r + c] = Rc[3 * r] * P.R[c] + Rc[3 * r + 1] * P.R[3 + c] + Rc[3 * r + 2] * P.R[6 + c];
    Pc.t[r] = Rc[3 * r] * P.t[0] + Rc[3 * r + 1] * P.t[1] + Rc[3 * r + 2] * P.t[2] + tc[r];
  }
}

// Rows of candidate slot `local` (index within the query) for every camera:
// K [R | t] with rows a and b divided by tau, as float4 x 4 per camera.
__device__ inline void write_candidate_rows(const QueryDesc& d, float* proj, int64_t local, const Pose& P) {
  const int rows = rows_per_slot(d);
  const double inv_tau = 1.0 / d.tau;
  for (int c = 0; c < rows; ++c) {
    Pose Pc;
    Cam K;
    camera_pose(d, c, P, Pc, K);
    double M[12];
    projection_rows(Pc, K, M);
    float4* pr = reinterpret_cast<float4*>(proj + d.proj_off + 16 * ((int64_t)rows * local + c));
    pr[0] = make_float4((float)(M[0] * inv_tau), (float)(M[1] * inv_tau), (float)(M[2] * inv_tau),
                        (float)(M[3] * inv_tau));
    pr[1] = make_float4((float)(M[4] * inv_tau), (float)(M[5] * inv_tau), (float)(M[6] * inv_tau),
                        (float)(M[7] * inv_tau));
    pr[2] = make_float4((float)M[8], (float)M[9], (float)M[10], (float)M[11]);
    pr[3] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

}  // namespace imloc
