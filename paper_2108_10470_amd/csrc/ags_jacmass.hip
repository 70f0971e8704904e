// Jacobian and joint-space inertia tensors of the environments of one model (Section 2.3: besides the
// state tensors, articulated actors expose Jacobian matrices and generalized mass matrices, per
// homogeneous group of actors, for operational-space control and inverse kinematics; Table 1).
//
// One 64-lane workgroup per environment, FP64 throughout (outputs FP32):
//   1. forward kinematics level by level (lanes over the links of a level): link rotation, origin,
//      world joint axis, world COM and world inertia about the COM, in LDS;
//   2. Jacobian: for every link b and generalized column k (lanes over k), the world velocity of b's
//      origin and b's world angular velocity per unit velocity of column k;
//   3. mass matrix: M[k][l] = sum over links b moved by both columns of
//      m_b vc_bk . vc_bl + w_bk . (I_b w_bl), with vc the velocity of b's COM and w the angular velocity
//      per unit column velocity: the kinetic energy 1/2 qd^T M qd written out body by body (lanes over
//      the (k, l) pairs with l >= k, mirrored).
// Column conventions are the step's: a free root contributes its world COM velocity (the root frame's
// origin is its COM) and its world angular velocity; every revolute or prismatic joint one rate.
#include <algorithm>

#include "ags_internal.h"

namespace ags {
namespace {

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ D3 ld(const double* p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ void st(double* p, D3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// row-major 3x3 times vector
__device__ __forceinline__ D3 mv(const double* R, D3 v) {
  return {R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
          R[6] * v.x + R[7] * v.y + R[8] * v.z};
}
// symmetric 3x3 stored xx yy zz xy xz yz, times vector
__device__ __forceinline__ D3 sv(const double* I, D3 v) {
  return {I[0] * v.x + I[3] * v.y + I[4] * v.z, I[3] * v.x + I[1] * v.y + I[5] * v.z,
          I[4] * v.x + I[5] * v.y + I[2] * v.z};
}
// rotation (row-major) of a unit quaternion xyzw
__device__ __forceinline__ void rot(const double* q, double* R) {
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w); R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w); R[7] = 2 * (y * z + x * w); R[8] = 1 - 2 * (x * x + y * y);
}

// per-link LDS arrays (FP64 words)
struct Kin {
  double *R, *q, *o, *ax, *c, *I;
};
__device__ __forceinline__ Kin kin_arrays(double* base, int nl) {
  Kin k;
  k.R = base;
  k.q = k.R + 9 * nl;
  k.o = k.q + 4 * nl;
  k.ax = k.o + 3 * nl;
  k.c = k.ax + 3 * nl;
  k.I = k.c + 3 * nl;
  return k;
}

// velocity (lin: of the world point `pt` carried by link b) and angular velocity of link b per unit rate
// of generalized column k; zero when column k does not move link b
__device__ __forceinline__ void column(const DevModel& M, const Kin& K, int b, int k, D3 pt, D3& lin, D3& ang) {
  lin = d3(0, 0, 0);
  ang = lin;
  const int j = M.col_link[k];
  if (!((M.link_anc[b] >> j) & 1ull)) return;
  const int* lj = M.li + j * LI_COLS;
  const int jt = lj[LI_JTYPE];
  const D3 arm = pt - ld(K.o + 3 * j);
  if (jt == J_FREE) {
    const int r = k - lj[LI_ROOTCOL];
    const D3 e = d3(r % 3 == 0 ? 1.0 : 0.0, r % 3 == 1 ? 1.0 : 0.0, r % 3 == 2 ? 1.0 : 0.0);
    if (r < 3) {
      lin = e;
    } else {
      ang = e;
      lin = cross(e, arm);
    }
  } else if (jt == J_REV) {
    ang = ld(K.ax + 3 * j);
    lin = cross(ang, arm);
  } else if (jt == J_PRI) {
    lin = ld(K.ax + 3 * j);
  }
}

__global__ __launch_bounds__(64) void jacmass_kernel(JacMassArgs A) {
  extern __shared__ double g_jm_lds[];
  const DevModel& M = A.m;
  const int nl = M.n_links, nv = M.n_v, lane = threadIdx.x;
  const int ei = blockIdx.x;
  if (ei >= A.n_envs) return;
  const int env = A.env_list[ei];
  const int abase = A.env_actor_base[env], dbase = A.env_dof_base[env], bbase = A.env_body_base[env];
  const Kin K = kin_arrays(g_jm_lds, nl);
  // 1. forward kinematics, one level at a time
  for (int lv = 0; lv < M.n_levels; ++lv) {
    for (int t = M.level_begin[lv] + lane; t < M.level_begin[lv + 1]; t += 64) {
      const int i = M.level_links[t];
      const int* li = M.li + i * LI_COLS;
      const double* lf = M.lf + i * LF_COLS;
      const int jt = li[LI_JTYPE];
      double* q = K.q + 4 * i;
      if (jt == J_FREE || jt == J_FIXED) {
        int a = 0;
        for (int k = 0; k < M.n_actors; ++k)
          if (M.ai[k * AI_COLS + AI_ROOT] == i) a = k;
        const float* rs = A.root_state + (long long)(abase + a) * 13;
        const double x = rs[3], y = rs[4], z = rs[5], w = rs[6];
        const double inv = 1.0 / sqrt(x * x + y * y + z * z + w * w);
        q[0] = x * inv; q[1] = y * inv; q[2] = z * inv; q[3] = w * inv;
        st(K.o + 3 * i, d3(rs[0], rs[1], rs[2]));
        st(K.ax + 3 * i, d3(0, 0, 0));
      } else {
        const int p = li[LI_PARENT];
        const double* qp = K.q + 4 * p;
        const D3 axl = ld(lf + LF_AXIS);
        D3 tl = ld(lf + LF_ANCHOR);
        const double qj = A.dof_state[(long long)(dbase + li[LI_DOF]) * 2];
        if (jt == J_REV) {  // parent orientation times the rotation by qj about the local axis
          const double sh = sin(0.5 * qj), ch = cos(0.5 * qj);
          const double rx = axl.x * sh, ry = axl.y * sh, rz = axl.z * sh;
          q[0] = qp[3] * rx + ch * qp[0] + (qp[1] * rz - qp[2] * ry);
          q[1] = qp[3] * ry + ch * qp[1] + (qp[2] * rx - qp[0] * rz);
          q[2] = qp[3] * rz + ch * qp[2] + (qp[0] * ry - qp[1] * rx);
          q[3] = qp[3] * ch - (qp[0] * rx + qp[1] * ry + qp[2] * rz);
        } else {
          for (int k = 0; k < 4; ++k) q[k] = qp[k];
          tl = tl + axl * qj;
        }
        const double* Rp = K.R + 9 * p;
        st(K.ax + 3 * i, mv(Rp, axl));
        st(K.o + 3 * i, ld(K.o + 3 * p) + mv(Rp, tl));
      }
      double* R = K.R + 9 * i;
      rot(q, R);
      st(K.c + 3 * i, ld(K.o + 3 * i) + mv(R, ld(lf + LF_COM)));
      // world inertia about the COM: R Ic R^T
      const double* ic = lf + LF_IC;
      const double Ic[9] = {ic[0], ic[3], ic[4], ic[3], ic[1], ic[5], ic[4], ic[5], ic[2]};
      double T[9];
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) T[3 * r + s] = R[3 * r] * Ic[s] + R[3 * r + 1] * Ic[3 + s] + R[3 * r + 2] * Ic[6 + s];
      auto e = [&](int r, int s) { return T[3 * r] * R[3 * s] + T[3 * r + 1] * R[3 * s + 1] + T[3 * r + 2] * R[3 * s + 2]; };
      double* I = K.I + 6 * i;
      I[0] = e(0, 0); I[1] = e(1, 1); I[2] = e(2, 2); I[3] = e(0, 1); I[4] = e(0, 2); I[5] = e(1, 2);
    }
    __syncthreads();
  }
  // 2. Jacobian (n_links x 6 x n_v per env)
  if (A.jac) {
    float* out = A.jac + (long long)ei * nl * 6 * nv;
    for (int b = 0; b < nl; ++b) {
      const D3 ob = ld(K.o + 3 * b);
      for (int k = lane; k < nv; k += 64) {
        D3 lin, ang;
        column(M, K, b, k, ob, lin, ang);
        float* o = out + (long long)b * 6 * nv + k;
        o[0] = (float)lin.x; o[nv] = (float)lin.y; o[2 * nv] = (float)lin.z;
        o[3 * nv] = (float)ang.x; o[4 * nv] = (float)ang.y; o[5 * nv] = (float)ang.z;
      }
    }
  }
  // 3. mass matrix (n_v x n_v per env), pairs l >= k
  if (A.mass) {
    float* out = A.mass + (long long)ei * nv * nv;
    for (int idx = lane; idx < nv * nv; idx += 64) {
      const int k = idx / nv, l = idx % nv;
      if (l < k) continue;
      const unsigned long long both = (1ull << M.col_link[k]) | (1ull << M.col_link[l]);
      double m = 0.0;
      for (int b = 0; b < nl; ++b) {
        if ((M.link_anc[b] & both) != both) continue;
        const D3 cb = ld(K.c + 3 * b);
        D3 vk, wk, vl, wl;
        column(M, K, b, k, cb, vk, wk);
        column(M, K, b, l, cb, vl, wl);
        const double sc = A.mass_scale ? double(A.mass_scale[bbase + b]) : 1.0;
        m += sc * (M.lf[b * LF_COLS + LF_MASS] * dot(vk, vl) + dot(wk, sv(K.I + 6 * b, wl)));
      }
      out[(long long)k * nv + l] = (float)m;
      out[(long long)l * nv + k] = (float)m;
    }
  }
}

}  // namespace

size_t jacmass_lds_bytes(int n_links) { return (size_t)28 * std::max(1, n_links) * sizeof(double); }

hipError_t launch_jacmass(const JacMassArgs& a, hipStream_t stream) {
  if (a.n_envs <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacmass_kernel, dim3(a.n_envs), dim3(64), jacmass_lds_bytes(a.m.n_links), stream, a);
  return hipGetLastError();
}

}  // namespace ags
