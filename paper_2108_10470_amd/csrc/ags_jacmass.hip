// Jacobian and joint-space inertia tensors of the environments of one model (Section 2.3: besides the
// state tensors, articulated actors expose Jacobian matrices and generalized mass matrices, per
// homogeneous group of actors, for operational-space control and inverse kinematics; Table 1).
//
// One 128-lane workgroup (two wavefronts) per environment, FP64 throughout (outputs FP32):
//   1. forward kinematics level by level (lanes over the links of a level): link rotation, origin and
//      world joint axis, in LDS;
//   2. composite inertias: every link's mass, first moment and rotational inertia about a reference
//      point (link 0's origin, which keeps the moments small), all links at once; then for every link j
//      the same terms summed over j's subtree (lanes over link and term);
//   3. per generalized column k: its spatial motion axis s_k = (w, v) at the reference point and the
//      momentum F_k = I^c s_k of the subtree the column moves (the composite-rigid-body form of M);
//   4. mass matrix: M[k][l] = s_l . F_k when l's link is an ancestor of (or is) k's link, the mirror
//      case likewise, and 0 for columns on unrelated branches (the kinetic energy 1/2 qd^T M qd summed
//      body by body, regrouped by subtree); each entry is computed from the ordered pair (min, max)
//      so that M is exactly symmetric;
//   5. Jacobian: for every link b and column k (lanes over the pairs), the world velocity of b's origin
//      and b's angular velocity per unit velocity of column k, from the column's spatial axis.
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
// rotation (row-major) of a unit quaternion xyzw
__device__ __forceinline__ void rot(const double* q, double* R) {
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w); R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w); R[7] = 2 * (y * z + x * w); R[8] = 1 - 2 * (x * x + y * y);
}

// per-link LDS arrays (FP64 words)
struct Kin {
  double *R, *q, *o, *ax;
};
__device__ __forceinline__ Kin kin_arrays(double* base, int nl) {
  Kin k;
  k.R = base;
  k.q = k.R + 9 * nl;
  k.o = k.q + 4 * nl;
  k.ax = k.o + 3 * nl;
  return k;
}

constexpr int kJmThreads = 128;

// Eight wavefronts per SIMD: at ~10 KB of LDS per env a CU holds fifteen workgroups, and the compiler's
// default register budget would admit only six wavefronts per SIMD (one FP64 register pair spills).
__global__ __launch_bounds__(kJmThreads) __attribute__((amdgpu_waves_per_eu(8))) void jacmass_kernel(JacMassArgs A) {
  extern __shared__ double g_jm_lds[];
  const DevModel& M = A.m;
  const int nl = M.n_links, nv = M.n_v, lane = threadIdx.x;
  const int ei = blockIdx.x;
  if (ei >= A.n_envs) return;
  const int env = A.env_list[ei];
  const int abase = A.env_actor_base[env], dbase = A.env_dof_base[env], bbase = A.env_body_base[env];
  const Kin K = kin_arrays(g_jm_lds, nl);
  double* const own = K.ax + 3 * nl; // per link: mass, first moment (3), rotational inertia (6) about the
  double* const cmp = own + 10 * nl; //   reference point; the same summed over the link's subtree
  double* const sc = cmp + 10 * nl;  // per column: motion axis w, v at the reference point (6)
  double* const fc = sc + 6 * nv;    // per column: momentum L, p (6)
  double* const qv = fc + 6 * nv;    // per link: joint position (0 for roots)
  unsigned long long* const anc = reinterpret_cast<unsigned long long*>(qv + nl);  // per link: ancestor mask
  int* const jtp = reinterpret_cast<int*>(anc + nl);        // per link: joint type | parent << 8
  int* const lvl = jtp + nl;                                 // links in level order
  int* const colk = lvl + nl;                                // per column: its link
  // 0. tables every later phase reads, staged once (independent loads spread over the lanes)
  for (int i = lane; i < nl; i += kJmThreads) {
    const int* li = M.li + i * LI_COLS;
    const int jt = li[LI_JTYPE];
    anc[i] = M.link_anc[i];
    jtp[i] = jt | (li[LI_PARENT] << 8);
    lvl[i] = M.level_links[i];
    qv[i] = (jt == J_FREE || jt == J_FIXED) ? 0.0 : double(A.dof_state[(long long)(dbase + li[LI_DOF]) * 2]);
  }
  for (int k = lane; k < nv; k += kJmThreads) colk[k] = M.col_link[k];
  __syncthreads();
  // 1. forward kinematics, one level at a time: only what a child needs of its parent
  for (int lv = 0; lv < M.n_levels; ++lv) {
    for (int t = M.level_begin[lv] + lane; t < M.level_begin[lv + 1]; t += kJmThreads) {
      const int i = lvl[t];
      const double* lf = M.lf + i * LF_COLS;
      const int jt = jtp[i] & 0xff;
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
        const int p = jtp[i] >> 8;
        const double* qp = K.q + 4 * p;
        const D3 axl = ld(lf + LF_AXIS);
        D3 tl = ld(lf + LF_ANCHOR);
        const double qj = qv[i];
        if (jt == J_REV) {  // parent orientation times the rotation by qj about the local axis
          double sh, chq;
          sincos(0.5 * qj, &sh, &chq);
          const double rx = axl.x * sh, ry = axl.y * sh, rz = axl.z * sh;
          q[0] = qp[3] * rx + chq * qp[0] + (qp[1] * rz - qp[2] * ry);
          q[1] = qp[3] * ry + chq * qp[1] + (qp[2] * rx - qp[0] * rz);
          q[2] = qp[3] * rz + chq * qp[2] + (qp[0] * ry - qp[1] * rx);
          q[3] = qp[3] * chq - (qp[0] * rx + qp[1] * ry + qp[2] * rz);
        } else {
          for (int k = 0; k < 4; ++k) q[k] = qp[k];
          tl = tl + axl * qj;
        }
        const double* Rp = K.R + 9 * p;
        st(K.ax + 3 * i, mv(Rp, axl));
        st(K.o + 3 * i, ld(K.o + 3 * p) + mv(Rp, tl));
      }
      rot(q, K.R + 9 * i);
    }
    __syncthreads();
  }
  const D3 ref = ld(K.o);
  if (A.mass) {
    // 2a. every link's own mass terms at once (lanes over links): mass f m, first moment f m c and
    //     rotational inertia f (R Ic R^T + m (|c|^2 1 - c c^T)) about the reference point, c its COM
    for (int i = lane; i < nl; i += kJmThreads) {
      const double* lf = M.lf + i * LF_COLS;
      const double* R = K.R + 9 * i;
      const double f = A.mass_scale ? double(A.mass_scale[bbase + i]) : 1.0;
      const double m = f * lf[LF_MASS];
      const D3 c = ld(K.o + 3 * i) + mv(R, ld(lf + LF_COM)) - ref;
      const double* ic = lf + LF_IC;
      const double Ic[9] = {ic[0], ic[3], ic[4], ic[3], ic[1], ic[5], ic[4], ic[5], ic[2]};
      double T[9];
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) T[3 * r + s] = R[3 * r] * Ic[s] + R[3 * r + 1] * Ic[3 + s] + R[3 * r + 2] * Ic[6 + s];
      auto e = [&](int r, int s) { return f * (T[3 * r] * R[3 * s] + T[3 * r + 1] * R[3 * s + 1] + T[3 * r + 2] * R[3 * s + 2]); };
      double* o = own + 10 * i;
      o[0] = m;
      o[1] = m * c.x; o[2] = m * c.y; o[3] = m * c.z;
      o[4] = e(0, 0) + m * (c.y * c.y + c.z * c.z);
      o[5] = e(1, 1) + m * (c.x * c.x + c.z * c.z);
      o[6] = e(2, 2) + m * (c.x * c.x + c.y * c.y);
      o[7] = e(0, 1) - m * c.x * c.y;
      o[8] = e(0, 2) - m * c.x * c.z;
      o[9] = e(1, 2) - m * c.y * c.z;
    }
    __syncthreads();
    // 2b. subtree sums, lanes over (link j, term): the bodies b whose ancestors include j
    for (int u = lane; u < 10 * nl; u += kJmThreads) {
      const int j = u / 10, c = u - 10 * j;
      double acc = 0.0;
      for (int b = 0; b < nl; ++b)
        if ((anc[b] >> j) & 1ull) acc += own[10 * b + c];
      cmp[u] = acc;
    }
    __syncthreads();
  }
  // 3. per column: motion axis at the reference point and (for M) the momentum of the subtree it moves
  for (int k = lane; k < nv; k += kJmThreads) {
    const int j = colk[k];
    const int* lj = M.li + j * LI_COLS;
    const int jt = lj[LI_JTYPE];
    const D3 oj = ld(K.o + 3 * j) - ref;
    D3 w = d3(0, 0, 0), v = w;
    if (jt == J_FREE) {
      const int r = k - lj[LI_ROOTCOL];
      const D3 e = d3(r % 3 == 0 ? 1.0 : 0.0, r % 3 == 1 ? 1.0 : 0.0, r % 3 == 2 ? 1.0 : 0.0);
      if (r < 3) {
        v = e;
      } else {
        w = e;
        v = cross(oj, e);
      }
    } else if (jt == J_REV) {
      w = ld(K.ax + 3 * j);
      v = cross(oj, w);
    } else if (jt == J_PRI) {
      v = ld(K.ax + 3 * j);
    }
    st(sc + 6 * k, w);
    st(sc + 6 * k + 3, v);
    if (A.mass) {  // momentum of the subtree: L = J w + h x v, p = m v + w x h
      const double* C = cmp + 10 * j;
      const D3 h = ld(C + 1);
      const double* J = C + 4;  // xx yy zz xy xz yz
      const D3 Jw = d3(J[0] * w.x + J[3] * w.y + J[4] * w.z, J[3] * w.x + J[1] * w.y + J[5] * w.z,
                       J[4] * w.x + J[5] * w.y + J[2] * w.z);
      st(fc + 6 * k, Jw + cross(h, v));
      st(fc + 6 * k + 3, v * C[0] + cross(w, h));
    }
  }
  __syncthreads();
  // 4. mass matrix, lanes over the flat output index
  if (A.mass) {
    float* out = A.mass + (long long)ei * nv * nv;
    for (int idx = lane; idx < nv * nv; idx += kJmThreads) {
      const int k0 = idx / nv, l0 = idx - k0 * nv;
      const int a = min(k0, l0), b = max(k0, l0);
      const int la = colk[a], lb = colk[b];
      int s = -1, f = -1;  // motion axis of the column on the ancestor link, momentum of the other
      if ((anc[lb] >> la) & 1ull) {
        s = a;
        f = b;
      } else if ((anc[la] >> lb) & 1ull) {
        s = b;
        f = a;
      }
      double m = 0.0;
      if (s >= 0) {
        const double* S = sc + 6 * s;
        const double* F = fc + 6 * f;
        m = S[0] * F[0] + S[1] * F[1] + S[2] * F[2] + S[3] * F[3] + S[4] * F[4] + S[5] * F[5];
      }
      out[idx] = (float)m;
    }
  }
  // 5. Jacobian (n_links x 6 x n_v per env), lanes over the (link b, column k) pairs: column k moves b
  //    iff k's link is an ancestor of b (or b itself); then b's origin moves at v_k + w_k x (o_b - ref)
  //    and b turns at w_k. Each pair writes its six rows, a wave's stores covering whole row runs.
  if (A.jac) {
    float* out = A.jac + (long long)ei * nl * 6 * nv;
    for (int pi = lane; pi < nl * nv; pi += kJmThreads) {
      const int b = pi / nv, k = pi - b * nv;
      D3 w = d3(0, 0, 0), lin = w;
      if ((anc[b] >> colk[k]) & 1ull) {
        const double* S = sc + 6 * k;
        w = ld(S);
        lin = ld(S + 3) + cross(w, ld(K.o + 3 * b) - ref);
      }
      float* o = out + (long long)b * 6 * nv + k;
      o[0] = (float)lin.x; o[nv] = (float)lin.y; o[2 * nv] = (float)lin.z;
      o[3 * nv] = (float)w.x; o[4 * nv] = (float)w.y; o[5 * nv] = (float)w.z;
    }
  }
}

}  // namespace

size_t jacmass_lds_bytes(int n_links, int n_v) {
  // per link: kinematics 19, own and subtree mass terms 20, q and ancestor mask 2, joint type and level
  // order 1; per column: axes and momenta 12, link 1
  return ((size_t)42 * std::max(1, n_links) + (size_t)13 * std::max(1, n_v)) * sizeof(double);
}

hipError_t launch_jacmass(const JacMassArgs& a, hipStream_t stream) {
  if (a.n_envs <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacmass_kernel, dim3(a.n_envs), dim3(kJmThreads), jacmass_lds_bytes(a.m.n_links, a.m.n_v), stream,
                     a);
  return hipGetLastError();
}

}  // namespace ags
