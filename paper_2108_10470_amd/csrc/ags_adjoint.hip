// Reverse-mode derivative of one env-step (hand-written adjoint), for gfx950: one wavefront per
// environment.
//
// The paper's simulator is not differentiable; this adjoint differentiates the step implemented
// by step_kernel (same readings: controls, free dynamics, speculative plane contacts and joint
// limits, fixed-sweep projected Gauss-Seidel, semi-implicit integration) with the discrete
// decisions (which rows exist, which bias branch and which clamp each Gauss-Seidel update took)
// held fixed, i.e. the derivative of the smooth piece the state lies in.
//
// Inputs: the state at the start of the step, its controls, and the adjoint of the state after
// the step.  The kernel recomputes the substeps (storing each substep's start state), then walks
// them backwards: recompute the substep with everything it needs in LDS, reverse it.
//
// The recomputation uses its own formulation, chosen so that every derivative is a short sweep
// over the tree: spatial vectors about a fixed reference point (the first actor's root position
// at the start of the step), world axes; M~ assembled from composite inertias and factored
// densely (Cholesky); C(q, qd) by the recursive Newton-Euler algorithm; row responses
// W = M~^-1 J^T by triangular solves.  In reverse:
//   * Gauss-Seidel is reversed row by row from a tape of (lambda before, lambda after, residual,
//     clamp state), giving the adjoints of the initial row velocities y0 = J v*, the biases and the
//     Delassus matrix A = J W (its diagonal through 1/A_rr);
//   * every term in which M~ is differentiated (through W, the impulse response W lambda and the
//     free accelerations) is gathered into one symmetric matrix P, and d tr(M P) / dq is taken in
//     one pass in CRBA form: sum_k 2 s_k^T Ic_k y_k + P_kk s_k^T Ic_k s_k with y_k the P-weighted
//     sum of the ancestor axes of column k;
//   * the velocity-product and gravity terms C(q, qd) are differentiated by reversing RNEA;
//   * each world quantity (axes, joint origins, centres of mass, inertias, contact points) receives
//     an adjoint; these become one wrench per link, and the subtree sums of the wrenches dotted
//     with the joint axes give the position adjoints (a free root: translation and the rotation
//     vector, mapped to the quaternion).
#include "ags_internal.h"

namespace ags {
static_assert(LI_COLS == kLinkIntCols, "the adjoint's staged link table and the model's link table differ in width");
namespace {

__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float min_(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double min_(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ void sincos_(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_(double x, double* s, double* c) { sincos(x, s, c); }

template <typename R>
struct V3 {
  R x, y, z;
};
template <typename R>
__device__ __forceinline__ V3<R> mk(R x, R y, R z) {
  return {x, y, z};
}
template <typename R>
__device__ __forceinline__ V3<R> zero3() {
  return {R(0), R(0), R(0)};
}
template <typename R>
__device__ __forceinline__ V3<R> add(V3<R> a, V3<R> b) {
  return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> sub(V3<R> a, V3<R> b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> mul(V3<R> a, R s) {
  return {a.x * s, a.y * s, a.z * s};
}
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename R, typename T>
__device__ __forceinline__ V3<R> ld3(const T* p) {
  return {R(p[0]), R(p[1]), R(p[2])};
}
template <typename R>
__device__ __forceinline__ void st3(R* p, V3<R> v) {
  p[0] = v.x;
  p[1] = v.y;
  p[2] = v.z;
}
template <typename R>
__device__ __forceinline__ void acc3(R* p, V3<R> v) {
  p[0] += v.x;
  p[1] += v.y;
  p[2] += v.z;
}
template <typename R>
__device__ __forceinline__ V3<R> mv(const R* M, V3<R> v) {
  return {M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
          M[6] * v.x + M[7] * v.y + M[8] * v.z};
}
// symmetric 3x3 stored xx yy zz xy xz yz
template <typename R>
__device__ __forceinline__ V3<R> symv(const R* S, V3<R> v) {
  return {S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
          S[4] * v.x + S[5] * v.y + S[2] * v.z};
}

// spatial vectors [angular; linear], linear parts about the reference point
template <typename R>
struct SV {
  V3<R> w, v;
};
template <typename R>
__device__ __forceinline__ SV<R> sz() {
  return {zero3<R>(), zero3<R>()};
}
template <typename R>
__device__ __forceinline__ SV<R> sadd(SV<R> a, SV<R> b) {
  return {add(a.w, b.w), add(a.v, b.v)};
}
template <typename R>
__device__ __forceinline__ SV<R> smul(SV<R> a, R s) {
  return {mul(a.w, s), mul(a.v, s)};
}
template <typename R>
__device__ __forceinline__ R sdot(SV<R> a, SV<R> b) {
  return dot(a.w, b.w) + dot(a.v, b.v);
}
// motion cross product V x m and force cross product V x* f
template <typename R>
__device__ __forceinline__ SV<R> crm(SV<R> V, SV<R> m) {
  return {cross(V.w, m.w), add(cross(V.w, m.v), cross(V.v, m.w))};
}
template <typename R>
__device__ __forceinline__ SV<R> crf(SV<R> V, SV<R> f) {
  return {add(cross(V.w, f.w), cross(V.v, f.v)), cross(V.w, f.v)};
}
template <typename R>
__device__ __forceinline__ SV<R> lds6(const R* p) {
  return {mk(p[0], p[1], p[2]), mk(p[3], p[4], p[5])};
}
template <typename R>
__device__ __forceinline__ void sts6(R* p, SV<R> a) {
  st3(p, a.w);
  st3(p + 3, a.v);
}
template <typename R>
__device__ __forceinline__ void acc6(R* p, SV<R> a) {
  acc3(p, a.w);
  acc3(p + 3, a.v);
}
// rigid body (mass m, COM c, inertia Iw about the COM) acting on a motion vector
template <typename R>
__device__ __forceinline__ SV<R> body_mul(R m, V3<R> c, const R* Iw, SV<R> X) {
  const V3<R> u = mul(add(X.v, cross(X.w, c)), m);
  return {add(symv(Iw, X.w), cross(c, u)), u};
}
// composite inertia [m, h = sum m c, J = sum (I + m (|c|^2 1 - c c^T)) as xx yy zz xy xz yz]
template <typename R>
__device__ __forceinline__ SV<R> comp_mul(const R* Ic, SV<R> X) {
  const V3<R> h = mk(Ic[1], Ic[2], Ic[3]);
  return {add(symv(Ic + 4, X.w), cross(h, X.v)), sub(mul(X.v, Ic[0]), cross(h, X.w))};
}
// adjoint of wgt <Y, I X> with respect to the body's COM (point) and orientation (torque)
template <typename R>
__device__ __forceinline__ void bil(R m, V3<R> c, const R* Iw, SV<R> Y, SV<R> X, R wgt, V3<R>& cb, V3<R>& tI) {
  const V3<R> uY = add(Y.v, cross(Y.w, c)), uX = add(X.v, cross(X.w, c));
  cb = add(cb, mul(add(cross(uY, X.w), cross(uX, Y.w)), wgt * m));
  tI = add(tI, mul(add(cross(symv(Iw, X.w), Y.w), cross(symv(Iw, Y.w), X.w)), wgt));
}

template <typename R>
__device__ __forceinline__ R wave_sum(R x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}
__device__ __forceinline__ unsigned long long lanes_below(int t) { return (1ull << t) - 1ull; }
__device__ __forceinline__ int lane_read(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float lane_read(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_read(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Hamilton product, xyzw
template <typename R>
__device__ __forceinline__ void qmul(const R* a, const R* b, R* o) {
  o[0] = a[3] * b[0] + a[0] * b[3] + a[1] * b[2] - a[2] * b[1];
  o[1] = a[3] * b[1] - a[0] * b[2] + a[1] * b[3] + a[2] * b[0];
  o[2] = a[3] * b[2] + a[0] * b[1] - a[1] * b[0] + a[2] * b[3];
  o[3] = a[3] * b[3] - a[0] * b[0] - a[1] * b[1] - a[2] * b[2];
}
// rotation increment Exp(theta) = (sin(|t|/2) t/|t|, cos(|t|/2)); (t/2, 1) below 1e-8
template <typename R>
__device__ __forceinline__ void dq_of(V3<R> th, R* dq) {
  const R ang = sqrt_(dot(th, th));
  if (ang < R(1e-8)) {
    dq[0] = R(0.5) * th.x; dq[1] = R(0.5) * th.y; dq[2] = R(0.5) * th.z; dq[3] = R(1);
  } else {
    R s, c;
    sincos_(R(0.5) * ang, &s, &c);
    const R sc = s / ang;
    dq[0] = th.x * sc; dq[1] = th.y * sc; dq[2] = th.z * sc; dq[3] = c;
  }
}
template <typename R>
__device__ __forceinline__ V3<R> dq_adj(V3<R> th, const R* dqb) {
  const R ang = sqrt_(dot(th, th));
  const V3<R> gv = mk(dqb[0], dqb[1], dqb[2]);
  if (ang < R(1e-8)) return mul(gv, R(0.5));
  R s, c;
  sincos_(R(0.5) * ang, &s, &c);
  const R sc = s / ang;
  const R dsc = (R(0.5) * c * ang - s) / (ang * ang);  // d(sin(a/2)/a)/da
  return add(mul(gv, sc), mul(th, (dot(th, gv) * dsc - R(0.5) * s * dqb[3]) / ang));
}

// tangent basis of a contact normal: t1 = normalised projection of the world axis least aligned with n
// (lowest index on ties), t2 = n x t1 (the rule of the step kernel)
template <typename R>
__device__ __forceinline__ int tangents(V3<R> n, V3<R>& t1, V3<R>& t2, V3<R>& t) {
  const R ax = n.x < R(0) ? -n.x : n.x, ay = n.y < R(0) ? -n.y : n.y, az = n.z < R(0) ? -n.z : n.z;
  int k = 0;
  R best = ax;
  if (ay < best) {
    best = ay;
    k = 1;
  }
  if (az < best) k = 2;
  const V3<R> e = k == 0 ? mk(R(1), R(0), R(0)) : (k == 1 ? mk(R(0), R(1), R(0)) : mk(R(0), R(0), R(1)));
  t = sub(e, mul(n, dot(n, e)));
  t1 = mul(t, R(1) / sqrt_(dot(t, t)));
  t2 = cross(n, t1);
  return k;
}
// adjoint of n through (t1, t2) = tangents(n)
template <typename R>
__device__ __forceinline__ V3<R> tangents_adj(V3<R> n, V3<R> t1b, V3<R> t2b) {
  V3<R> t1, t2, t;
  const int k = tangents(n, t1, t2, t);
  V3<R> nb = cross(t1, t2b);
  t1b = add(t1b, cross(t2b, n));
  const V3<R> tb = mul(sub(t1b, mul(t1, dot(t1, t1b))), R(1) / sqrt_(dot(t, t)));
  const R nk = k == 0 ? n.x : (k == 1 ? n.y : n.z);
  nb = sub(nb, mul(tb, nk));
  const R ntb = dot(n, tb);
  if (k == 0) nb.x -= ntb;
  else if (k == 1) nb.y -= ntb;
  else nb.z -= ntb;
  return nb;
}
// sphere (centre c, radius r) against a box (rotation Rb row-major, centre b, half extents hb): signed
// distance and normal (from the box towards the sphere) by the closest point, or the face of least
// penetration when the centre is inside (the step kernel's rule).  G (optional) = dn / d(c - moving box
// point), row-major: Rb (1 - nl nl^T) diag(clamped axes) Rb^T / |d| outside, 0 inside.
template <typename R>
__device__ __forceinline__ void sphere_box(V3<R> c, const R* Rb, V3<R> b, V3<R> hb, R rad, R& phi, V3<R>& n, R* G) {
  const V3<R> u = sub(c, b);
  const V3<R> xl = mk(Rb[0] * u.x + Rb[3] * u.y + Rb[6] * u.z, Rb[1] * u.x + Rb[4] * u.y + Rb[7] * u.z,
                      Rb[2] * u.x + Rb[5] * u.y + Rb[8] * u.z);
  const V3<R> ql = mk(fmin(fmax(xl.x, -hb.x), hb.x), fmin(fmax(xl.y, -hb.y), hb.y), fmin(fmax(xl.z, -hb.z), hb.z));
  const bool inside = ql.x == xl.x && ql.y == xl.y && ql.z == xl.z;
  const V3<R> dl = sub(xl, ql);
  const R dn = sqrt_(dot(dl, dl));
  V3<R> nl;
  if (!inside && dn > R(1e-12)) {
    phi = dn - rad;
    nl = mul(dl, R(1) / dn);
    if (G) {
      const R m[3] = {xl.x != ql.x ? R(1) : R(0), xl.y != ql.y ? R(1) : R(0), xl.z != ql.z ? R(1) : R(0)};
      const R nv[3] = {nl.x, nl.y, nl.z};
      R Lc[9];  // (1 - nl nl^T) diag(m) / dn in box coordinates
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Lc[3 * i + j] = ((i == j ? R(1) : R(0)) - nv[i] * nv[j]) * m[j] / dn;
      R T[9];  // Rb Lc
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) T[3 * i + j] = Rb[3 * i] * Lc[j] + Rb[3 * i + 1] * Lc[3 + j] + Rb[3 * i + 2] * Lc[6 + j];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[3 * i + j] = T[3 * i] * Rb[3 * j] + T[3 * i + 1] * Rb[3 * j + 1] + T[3 * i + 2] * Rb[3 * j + 2];
    }
  } else {
    const R p0 = hb.x - (xl.x < R(0) ? -xl.x : xl.x), p1 = hb.y - (xl.y < R(0) ? -xl.y : xl.y),
            p2 = hb.z - (xl.z < R(0) ? -xl.z : xl.z);
    int kb = 0;
    R pb = p0, xb = xl.x;
    if (p1 < pb) { kb = 1; pb = p1; xb = xl.y; }
    if (p2 < pb) { kb = 2; pb = p2; xb = xl.z; }
    const R sg = xb >= R(0) ? R(1) : R(-1);
    nl = kb == 0 ? mk(sg, R(0), R(0)) : (kb == 1 ? mk(R(0), sg, R(0)) : mk(R(0), R(0), sg));
    phi = -pb - rad;
    if (G) {
#pragma unroll
      for (int k = 0; k < 9; ++k) G[k] = R(0);
    }
  }
  n = mv(Rb, nl);
}

// packed symmetric storage: element (i, j) of a symmetric matrix
__device__ __forceinline__ int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }
// start of row i of a packed lower triangle (entries (i, j), j <= i)
__device__ __forceinline__ int lrow(int i) { return i * (i + 1) / 2; }

// ---------------------------------------------------------------- wavefront GEMM on the matrix cores
// C = X Y (M x N, inner dimension K, each at most 64) by one wavefront with 16x16x4 MFMA tiles.  x(i, k)
// and y(k, j) return operand entries (called only inside the bounds); out(i, j, c) receives each entry of C.
// Operand lanes: lane l supplies X[m0 + l % 16][k0 + l / 16] and Y[k0 + l / 16][n0 + l % 16]; result
// value v of lane l is row 4 (l / 16) + v (FP32) or 4 v + l / 16 (FP64) of the tile, column l % 16.
// Call from uniform control flow (all 64 lanes active).
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <typename R, typename FX, typename FY, typename FO>
__device__ __forceinline__ void wave_gemm(int M, int N, int K, int lane, const FX& x, const FY& y, const FO& out) {
  using T = Mfma<R>;
  const int lc = lane & 15, lk = lane >> 4;
  for (int m0 = 0; m0 < M; m0 += 16)
    for (int n0 = 0; n0 < N; n0 += 16) {
      typename T::v4 c = {R(0), R(0), R(0), R(0)};
      for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        const R a = (m0 + lc < M && k < K) ? x(m0 + lc, k) : R(0);
        const R b = (k < K && n0 + lc < N) ? y(k, n0 + lc) : R(0);
        c = T::step(a, b, c);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + T::row(lane, v), j = n0 + lc;
        if (i < M && j < N) out(i, j, c[v]);
      }
    }
}

// ---------------------------------------------------------------- per-environment context
// per-phase clock counters of the debug accounting, then the current phase and the last mark (lane 0)
__shared__ long long g_adj_clock[kAdjPhases + 2];

template <typename R>
struct Env {
  const AdjArgs* P;
  R* r;      // LDS reals of this environment
  int* ix;   // LDS ints
  int lane;
  int nl, nv, nd, na, ns, nlev, rc;
  int abase, dbase;
  R h;
  V3<R> g, ref;
  int R_;    // rows of the current substep
  // per-phase shader-clock accounting, only when the debug tensor is bound: the counters, the current phase
  // and the last mark live in LDS (g_adj_clock), so that no register is held for them through the kernel
  __device__ __forceinline__ void phase(int ph) {
    if (!P->cycles) return;
    if (lane == 0) {
      const long long now = (long long)clock64();
      const int cur = (int)g_adj_clock[kAdjPhases];
      if (cur >= 0) g_adj_clock[cur] += now - g_adj_clock[kAdjPhases + 1];
      g_adj_clock[kAdjPhases] = ph;
      g_adj_clock[kAdjPhases + 1] = now;
    }
  }
  // table access
  // the model's integer tables: staged in LDS by adjoint_env in the FP64 forms, read through the caches in the
  // FP32 forms (whose small layout would lose a workgroup per CU to them)
  static constexpr bool kStaged = sizeof(R) == 8;
  __device__ const int* li(int i) const { return (kStaged ? ix + P->L.t_li : P->m.li) + i * LI_COLS; }
  __device__ int lev_begin(int d) const { return kStaged ? ix[P->L.t_lev + d] : P->m.level_begin[d]; }
  __device__ int lev_link(int t) const { return kStaged ? ix[P->L.t_links + t] : P->m.level_links[t]; }
  __device__ int child(int k) const { return kStaged ? ix[P->L.t_child + k] : P->m.children[k]; }
  __device__ int col_link(int c) const { return kStaged ? ix[P->L.t_col + c] : P->m.col_link[c]; }
  __device__ int dof_link(int j) const { return kStaged ? ix[P->L.t_dof + j] : P->m.dof_link[j]; }
  __device__ const double* lf(int i) const { return P->m.lf + i * LF_COLS; }
  __device__ R* at(int off, int i, int w) const { return r + off + i * w; }
};

// One inward step of a children gather: every link of tree level lev adds its children's W-word records
// (at off, one per link) to its own, with lanes over (link, word) pairs instead of one lane walking a link's
// children record by record (the same sums in the same order).
template <typename R, int W>
__device__ __forceinline__ void gather_children_level(const Env<R>& E, int off, int lev) {
  const auto& M = E.P->m;
  const int b = E.lev_begin(lev), n_at = E.lev_begin(lev + 1) - b;
  for (int pi = E.lane; pi < n_at * W; pi += 64) {
    const int slot = pi / W, w = pi - slot * W;
    const int i = E.lev_link(b + slot);
    const int* li = E.li(i);
    R acc = E.r[off + i * W + w];
    for (int k = li[LI_CHILD_BEGIN]; k < li[LI_CHILD_END]; ++k) acc += E.r[off + E.child(k) * W + w];
    E.r[off + i * W + w] = acc;
  }
}

template <typename R>
__device__ __forceinline__ void sync() {
  __syncthreads();
}

// joint motion vector of link i (world axis ax, joint origin p)
template <typename R>
__device__ __forceinline__ SV<R> joint_s(const Env<R>& E, int i) {
  const AdjLds& L = E.P->L;
  const V3<R> ax = ld3<R>(E.at(L.ax, i, 3));
  if (E.li(i)[LI_JTYPE] == J_REV) return {ax, cross(ld3<R>(E.at(L.p, i, 3)), ax)};
  return {zero3<R>(), ax};
}
// motion vector of generalized column k (a joint's, or one of a free root's six), from geometry
template <typename R>
__device__ __forceinline__ SV<R> col_s_geo(const Env<R>& E, int k) {
  const int i = E.col_link(k);
  const int* li = E.li(i);
  if (li[LI_PARENT] >= 0) return joint_s(E, i);
  const int a = k - li[LI_ROOTCOL];
  V3<R> e = zero3<R>();
  if ((a % 3) == 0) e.x = R(1);
  else if ((a % 3) == 1) e.y = R(1);
  else e.z = R(1);
  if (a < 3) return {zero3<R>(), e};
  return {e, cross(ld3<R>(E.at(E.P->L.c, i, 3)), e)};
}
// the same, as stored once per substep after the kinematics
template <typename R>
__device__ __forceinline__ SV<R> col_s(const Env<R>& E, int k) {
  return lds6(E.r + E.P->L.cs + 6 * k);
}

// S_0 x for a free root with COM c0: (x_w, x_v + c0 x x_w)
template <typename R>
__device__ __forceinline__ SV<R> root_vel(V3<R> c0, const R* x) {
  const V3<R> v = mk(x[0], x[1], x[2]), w = mk(x[3], x[4], x[5]);
  return {w, add(v, cross(c0, w))};
}

// outward sweep: spatial velocity of every link under the generalized vector x (LDS, per column)
template <typename R>
__device__ void link_vel(const Env<R>& E, const R* x, int out) {
  const AdjLds& L = E.P->L;
  const DevModel& M = E.P->m;
  for (int lev = 0; lev < E.nlev; ++lev) {
    const int b = E.lev_begin(lev), e = E.lev_begin(lev + 1);
    for (int t = b + E.lane; t < e; t += 64) {
      const int i = E.lev_link(t);
      const int* li = E.li(i);
      SV<R> V;
      if (li[LI_PARENT] < 0) {
        V = li[LI_JTYPE] == J_FREE ? root_vel(ld3<R>(E.at(L.c, i, 3)), x + li[LI_ROOTCOL]) : sz<R>();
      } else {
        V = sadd(lds6(E.at(out, li[LI_PARENT], 6)), smul(joint_s(E, i), x[li[LI_COL]]));
      }
      sts6(E.at(out, i, 6), V);
    }
    sync<R>();
  }
}

// solve M~ x = b for one vector, lane c holding b_c (returns x_c); Lm holds the Cholesky factor
template <typename R>
__device__ R chol_solve_lanes(const Env<R>& E, R b) {
  const R* Lm = E.r + E.P->L.Lm;
  const R* ldi = E.r + E.P->L.ldi;
  const int nv = E.nv, c = E.lane;
  for (int k = 0; k < nv; ++k) {
    const R xk = lane_read(b, k) * ldi[k];
    if (c == k) b = xk;
    if (c > k && c < nv) b -= Lm[lrow(c) + k] * xk;
  }
  for (int k = nv - 1; k >= 0; --k) {
    const R xk = lane_read(b, k) * ldi[k];
    if (c == k) b = xk;
    if (c < k) b -= Lm[lrow(k) + c] * xk;
  }
  return c < nv ? b : R(0);
}
// solve in place on one LDS row per lane (row pointer y, length nv); four partial sums per dot product
constexpr int kRegSolve = 32;  // models with at most this many columns solve a row in registers

template <typename R>
__device__ void chol_solve_row(const Env<R>& E, R* y) {
  const R* Lm = E.r + E.P->L.Lm;
  const R* ldi = E.r + E.P->L.ldi;
  const int nv = E.nv;
  if (nv <= kRegSolve) {
    // the lane's row in registers: the substitutions' chains run through registers instead of a store and a
    // load of every solved entry (entries past n_v are zero and their factor reads are masked)
    R v[kRegSolve];
#pragma unroll
    for (int k = 0; k < kRegSolve; ++k) v[k] = k < nv ? y[k] : R(0);
#pragma unroll
    for (int k = 0; k < kRegSolve; ++k) {
      if (k < nv) {
        const R* Lk = Lm + lrow(k);
        R t[4] = {v[k], R(0), R(0), R(0)};
#pragma unroll
        for (int j = 0; j < k; ++j) t[j & 3] -= Lk[j] * v[j];
        v[k] = ((t[0] + t[1]) + (t[2] + t[3])) * ldi[k];
      }
    }
#pragma unroll
    for (int k = kRegSolve - 1; k >= 0; --k) {
      if (k < nv) {
        R t[4] = {v[k], R(0), R(0), R(0)};
#pragma unroll
        for (int j = k + 1; j < kRegSolve; ++j) {
          const R l = Lm[lrow(min(j, nv - 1)) + k];
          t[j & 3] -= (j < nv ? l : R(0)) * v[j];
        }
        v[k] = ((t[0] + t[1]) + (t[2] + t[3])) * ldi[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kRegSolve; ++k)
      if (k < nv) y[k] = v[k];
    return;
  }
  for (int k = 0; k < nv; ++k) {
    const R* Lk = Lm + lrow(k);
    R t0 = y[k], t1 = R(0), t2 = R(0), t3 = R(0);
    int j = 0;
    for (; j + 3 < k; j += 4) {
      t0 -= Lk[j] * y[j];
      t1 -= Lk[j + 1] * y[j + 1];
      t2 -= Lk[j + 2] * y[j + 2];
      t3 -= Lk[j + 3] * y[j + 3];
    }
    for (; j < k; ++j) t0 -= Lk[j] * y[j];
    y[k] = ((t0 + t1) + (t2 + t3)) * ldi[k];
  }
  for (int k = nv - 1; k >= 0; --k) {
    R t0 = y[k], t1 = R(0), t2 = R(0), t3 = R(0);
    int j = k + 1;
    for (; j + 3 < nv; j += 4) {
      t0 -= Lm[lrow(j) + k] * y[j];
      t1 -= Lm[lrow(j + 1) + k] * y[j + 1];
      t2 -= Lm[lrow(j + 2) + k] * y[j + 2];
      t3 -= Lm[lrow(j + 3) + k] * y[j + 3];
    }
    for (; j < nv; ++j) t0 -= Lm[lrow(j) + k] * y[j];
    y[k] = ((t0 + t1) + (t2 + t3)) * ldi[k];
  }
}

// ---------------------------------------------------------------- forward substep (recompute)
// sin: state at the start of the substep; sout: state after it.  Returns false when the substep
// has more constraint rows than the adjoint handles (wave-uniform).
template <typename R>
__device__ __forceinline__ bool fwd_substep(Env<R>& E, const R* sin, R* sout) {
  const AdjArgs& P = *E.P;
  const AdjLds& L = P.L;
  const DevModel& M = P.m;
  const int lane = E.lane, nv = E.nv, nd = E.nd, na = E.na;
  const R h = E.h;
  R* nu = E.r + L.nu;
  R* tau = E.r + L.tau;
  R* arm = E.r + L.arm;
  R* q = E.r + L.q;
  E.phase(0);
  // ---- controls, generalized velocity
  for (int c = lane; c < nv; c += 64) {
    tau[c] = R(0);
    arm[c] = R(0);
  }
  sync<R>();
  for (int a = lane; a < na; a += 64) {
    const int* ai = M.ai + a * AI_COLS;
    if (ai[AI_FIXED]) continue;
    const int c = ai[AI_COL];
    for (int k = 0; k < 6; ++k) nu[c + k] = sin[13 * a + 7 + k];
  }
  for (int j = lane; j < nd; j += 64) {
    const int i = E.dof_link(j);
    const int c = E.li(i)[LI_COL];
    const double* lf = E.lf(i);
    const R qj = sin[13 * na + 2 * j], qdj = sin[13 * na + 2 * j + 1];
    q[j] = qj;
    nu[c] = qdj;
    const R pt = P.pos_tgt ? R(P.pos_tgt[E.dbase + j]) : R(0);
    const R vt = P.vel_tgt ? R(P.vel_tgt[E.dbase + j]) : R(0);
    const R kp = R(lf[LF_KP]), kd = R(lf[LF_KD]);
    tau[c] = R(P.act[E.dbase + j]) + kp * (pt - qj - h * qdj) + kd * (vt - qdj);
    arm[c] = R(lf[LF_ARM]) + h * kd + h * h * kp;
  }
  sync<R>();
  // ---- joint-local rotation, anchor and axis of every link at once (lanes over links): they need only the
  // link's own joint coordinate, so the sines and cosines are not taken one tree level after the other.
  // Staged in the link's own Rm, p and ax words, which the level loop below overwrites with world values.
  for (int i = lane; i < E.nl; i += 64) {
    const int* li = E.li(i);
    if (li[LI_PARENT] < 0) continue;
    const double* lf = E.lf(i);
    const V3<R> axl = ld3<R>(lf + LF_AXIS);
    V3<R> tl = ld3<R>(lf + LF_ANCHOR);
    const R qi = q[li[LI_DOF]];
    R* Rr = E.at(L.Rm, i, 9);
    if (li[LI_JTYPE] == J_REV) {
      R s, c;
      sincos_(qi, &s, &c);
      const R t1 = R(1) - c;
      Rr[0] = c + t1 * axl.x * axl.x; Rr[1] = t1 * axl.x * axl.y - s * axl.z; Rr[2] = t1 * axl.x * axl.z + s * axl.y;
      Rr[3] = t1 * axl.x * axl.y + s * axl.z; Rr[4] = c + t1 * axl.y * axl.y; Rr[5] = t1 * axl.y * axl.z - s * axl.x;
      Rr[6] = t1 * axl.x * axl.z - s * axl.y; Rr[7] = t1 * axl.y * axl.z + s * axl.x; Rr[8] = c + t1 * axl.z * axl.z;
    } else {
      tl = add(tl, mul(axl, qi));
    }
    st3(E.at(L.p, i, 3), tl);
    st3(E.at(L.ax, i, 3), axl);
  }
  sync<R>();
  // ---- kinematics and velocities (outward by level); then every link's COM, world inertia and own
  // composite inertia at once (lanes over links): they need only the link's own pose
  for (int lev = 0; lev < E.nlev; ++lev) {
    const int b = E.lev_begin(lev), e = E.lev_begin(lev + 1);
    for (int t = b + lane; t < e; t += 64) {
      const int i = E.lev_link(t);
      const int* li = E.li(i);
      const double* lf = E.lf(i);
      R* Rm = E.at(L.Rm, i, 9);
      V3<R> pw;
      SV<R> V;
      if (li[LI_PARENT] < 0) {
        int a = 0;
        while (M.ai[a * AI_COLS + AI_ROOT] != i) ++a;
        const R* rs = sin + 13 * a;
        R qx = rs[3], qy = rs[4], qz = rs[5], qw = rs[6];
        const R inv = R(1) / sqrt_(qx * qx + qy * qy + qz * qz + qw * qw);
        qx *= inv; qy *= inv; qz *= inv; qw *= inv;
        Rm[0] = R(1) - R(2) * (qy * qy + qz * qz); Rm[1] = R(2) * (qx * qy - qz * qw); Rm[2] = R(2) * (qx * qz + qy * qw);
        Rm[3] = R(2) * (qx * qy + qz * qw); Rm[4] = R(1) - R(2) * (qx * qx + qz * qz); Rm[5] = R(2) * (qy * qz - qx * qw);
        Rm[6] = R(2) * (qx * qz - qy * qw); Rm[7] = R(2) * (qy * qz + qx * qw); Rm[8] = R(1) - R(2) * (qx * qx + qy * qy);
        pw = sub(ld3<R>(rs), E.ref);
        st3(E.at(L.ax, i, 3), zero3<R>());
      } else {
        // the staged joint-local parts (read whole before this link's words are overwritten)
        const int p = li[LI_PARENT];
        const R* Rp = E.at(L.Rm, p, 9);
        const V3<R> axl = ld3<R>(E.at(L.ax, i, 3));
        const V3<R> tl = ld3<R>(E.at(L.p, i, 3));
        if (li[LI_JTYPE] == J_REV) {
          R Rr[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) Rr[k] = Rm[k];
#pragma unroll
          for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
            for (int c0 = 0; c0 < 3; ++c0)
              Rm[3 * r0 + c0] = Rp[3 * r0] * Rr[c0] + Rp[3 * r0 + 1] * Rr[3 + c0] + Rp[3 * r0 + 2] * Rr[6 + c0];
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) Rm[k] = Rp[k];
        }
        st3(E.at(L.ax, i, 3), mv(Rp, axl));
        pw = add(ld3<R>(E.at(L.p, p, 3)), mv(Rp, tl));
      }
      st3(E.at(L.p, i, 3), pw);
      // velocity (a free root's needs its COM, the root frame's origin)
      if (li[LI_PARENT] < 0) {
        V = li[LI_JTYPE] == J_FREE ? root_vel(add(pw, mv(Rm, ld3<R>(lf + LF_COM))), nu + li[LI_ROOTCOL]) : sz<R>();
      } else {
        V = sadd(lds6(E.at(L.V, li[LI_PARENT], 6)), smul(joint_s(E, i), nu[li[LI_COL]]));
      }
      sts6(E.at(L.V, i, 6), V);
    }
    sync<R>();
  }
  for (int i = lane; i < E.nl; i += 64) {
    const double* lf = E.lf(i);
    const R* Rm = E.at(L.Rm, i, 9);
    // COM and world inertia
    const V3<R> cw = add(ld3<R>(E.at(L.p, i, 3)), mv(Rm, ld3<R>(lf + LF_COM)));
    st3(E.at(L.c, i, 3), cw);
    const R I0[9] = {R(lf[LF_IC + 0]), R(lf[LF_IC + 3]), R(lf[LF_IC + 4]), R(lf[LF_IC + 3]), R(lf[LF_IC + 1]),
                     R(lf[LF_IC + 5]), R(lf[LF_IC + 4]), R(lf[LF_IC + 5]), R(lf[LF_IC + 2])};
    R T[9];  // Rm I0
#pragma unroll
    for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
      for (int c0 = 0; c0 < 3; ++c0) T[3 * r0 + c0] = Rm[3 * r0] * I0[c0] + Rm[3 * r0 + 1] * I0[3 + c0] + Rm[3 * r0 + 2] * I0[6 + c0];
    R* Iw = E.at(L.Iw, i, 6);
    auto TRt = [&](int a, int b2) { return T[3 * a] * Rm[3 * b2] + T[3 * a + 1] * Rm[3 * b2 + 1] + T[3 * a + 2] * Rm[3 * b2 + 2]; };
    Iw[0] = TRt(0, 0); Iw[1] = TRt(1, 1); Iw[2] = TRt(2, 2); Iw[3] = TRt(0, 1); Iw[4] = TRt(0, 2); Iw[5] = TRt(1, 2);
    // own part of the composite inertia
    const R m = R(lf[LF_MASS]);
    R* Ic = E.at(L.Ic, i, 10);
    Ic[0] = m; Ic[1] = m * cw.x; Ic[2] = m * cw.y; Ic[3] = m * cw.z;
    const R cc = dot(cw, cw);
    Ic[4] = Iw[0] + m * (cc - cw.x * cw.x); Ic[5] = Iw[1] + m * (cc - cw.y * cw.y); Ic[6] = Iw[2] + m * (cc - cw.z * cw.z);
    Ic[7] = Iw[3] - m * cw.x * cw.y; Ic[8] = Iw[4] - m * cw.x * cw.z; Ic[9] = Iw[5] - m * cw.y * cw.z;
  }
  sync<R>();
  E.phase(8);
  // ---- composite inertias (inward by level, children gathered)
  for (int lev = E.nlev - 2; lev >= 0; --lev) {
    gather_children_level<R, 10>(E, L.Ic, lev);
    sync<R>();
  }
  for (int k = lane; k < nv; k += 64) sts6(E.r + L.cs + 6 * k, col_s_geo(E, k));
  sync<R>();
  // ---- M~ (lower triangle) from composite inertias: M_kj = s_j . (Ic_k s_k), j an ancestor column of k
  R* Lm = E.r + L.Lm;
  const int nvp = L.nvp;
  for (int k = lane; k < nv; k += 64) {
    const SV<R> sk = col_s(E, k);
    const SV<R> F = comp_mul(E.at(L.Ic, E.col_link(k), 10), sk);
    const unsigned long long anc = M.col_anc[k];
    for (int j = 0; j < k; ++j) Lm[lrow(k) + j] = ((anc >> j) & 1ull) ? sdot(col_s(E, j), F) : R(0);
    Lm[lrow(k) + k] = sdot(sk, F) + arm[k];
  }
  sync<R>();
  // ---- dense Cholesky in place, left-looking: column k from the finished columns j < k (lane = row)
  for (int k = 0; k < nv; ++k) {
    R sacc = R(0);
    if (lane >= k && lane < nv) {
      const R* Li = Lm + lrow(lane);
      const R* Lk = Lm + lrow(k);
      R t0 = Li[k], t1 = R(0), t2 = R(0), t3 = R(0);
      int j = 0;
      for (; j + 3 < k; j += 4) {
        t0 -= Li[j] * Lk[j];
        t1 -= Li[j + 1] * Lk[j + 1];
        t2 -= Li[j + 2] * Lk[j + 2];
        t3 -= Li[j + 3] * Lk[j + 3];
      }
      for (; j < k; ++j) t0 -= Li[j] * Lk[j];
      sacc = (t0 + t1) + (t2 + t3);
    }
    const R d = sqrt_(lane_read(sacc, k));
    const R di = R(1) / d;
    if (lane >= k && lane < nv) Lm[lrow(lane) + k] = lane == k ? d : sacc * di;
    if (lane == 0) E.r[L.ldi + k] = di;
    sync<R>();
  }
  E.phase(0);
  // ---- C(q, qd): RNEA with zero joint accelerations, gravity as a base acceleration
  for (int lev = 0; lev < E.nlev; ++lev) {
    const int b = E.lev_begin(lev), e = E.lev_begin(lev + 1);
    for (int t = b + lane; t < e; t += 64) {
      const int i = E.lev_link(t);
      const int* li = E.li(i);
      SV<R> A;
      if (li[LI_PARENT] < 0) {
        A = {zero3<R>(), mul(E.g, R(-1))};
        if (li[LI_JTYPE] == J_FREE) {
          const R* x = nu + li[LI_ROOTCOL];
          A.v = add(A.v, cross(mk(x[0], x[1], x[2]), mk(x[3], x[4], x[5])));
        }
      } else {
        A = sadd(lds6(E.at(L.X1, li[LI_PARENT], 6)), smul(crm(lds6(E.at(L.V, li[LI_PARENT], 6)), joint_s(E, i)), nu[li[LI_COL]]));
      }
      sts6(E.at(L.X1, i, 6), A);
    }
    sync<R>();
  }
  // body forces of every link at once: they need only its own acceleration and velocity
  for (int i = lane; i < E.nl; i += 64) {
    const SV<R> A = lds6(E.at(L.X1, i, 6));
    const R m = R(E.lf(i)[LF_MASS]);
    const V3<R> cw = ld3<R>(E.at(L.c, i, 3));
    const R* Iw = E.at(L.Iw, i, 6);
    const SV<R> V = lds6(E.at(L.V, i, 6));
    sts6(E.at(L.X2, i, 6), sadd(body_mul(m, cw, Iw, A), crf(V, body_mul(m, cw, Iw, V))));
  }
  sync<R>();
  for (int lev = E.nlev - 2; lev >= 0; --lev) {
    gather_children_level<R, 6>(E, L.X2, lev);
    sync<R>();
  }
  R rhs = R(0);
  if (lane < nv) {
    const int i = E.col_link(lane);
    const int* li = E.li(i);
    const SV<R> F = lds6(E.at(L.X2, i, 6));
    R C;
    if (li[LI_PARENT] >= 0) {
      C = sdot(joint_s(E, i), F);
    } else {
      const int a = lane - li[LI_ROOTCOL];
      const V3<R> n0 = add(F.w, cross(F.v, ld3<R>(E.at(L.c, i, 3))));
      C = a == 0 ? F.v.x : a == 1 ? F.v.y : a == 2 ? F.v.z : a == 3 ? n0.x : a == 4 ? n0.y : n0.z;
    }
    rhs = tau[lane] - C;
  }
  const R qddc = chol_solve_lanes(E, rhs);
  R* vs = E.r + L.vs;
  if (lane < nv) {
    E.r[L.qdd + lane] = qddc;
    vs[lane] = nu[lane] + h * qddc;
  }
  sync<R>();
  link_vel(E, vs, L.Vs);
  // ---- rows: joint limits (by DOF, lower before upper), then plane contacts (slot order; n, t1, t2)
  int* rkind = E.ix + L.rkind;
  int* rlink = E.ix + L.rlink;
  int* rdof = E.ix + L.rdof;
  int* rnrm = E.ix + L.rnrm;
  R* rbc = E.r + L.rbc;
  R* rb = E.r + L.rb;
  R* rx = E.r + L.rx;
  R* rcen = E.r + L.rcen;
  R* rd = E.r + L.rd;
  const int rcap = E.rc;
  int nrows = 0;
  {
    bool alo = false, ahi = false;
    R glo = R(0), ghi = R(0);
    int i = 0;
    if (lane < nd) {
      i = E.dof_link(lane);
      const double* lf = E.lf(i);
      const R lo = R(lf[LF_LO]), hi = R(lf[LF_HI]), ml = R(lf[LF_ML]);
      const R rate = vs[E.li(i)[LI_COL]];
      glo = q[lane] - lo;
      ghi = hi - q[lane];
      alo = isfinite(lf[LF_LO]) && min_(glo, glo + h * rate) < ml;
      ahi = isfinite(lf[LF_HI]) && min_(ghi, ghi - h * rate) < ml;
    }
    const unsigned long long mlo = __ballot(alo), mhi = __ballot(ahi);
    const unsigned long long below = lanes_below(lane);
    const int base = __popcll(mlo & below) + __popcll(mhi & below);
    nrows = __popcll(mlo) + __popcll(mhi);
    if (alo && base < rcap) {
      rkind[base] = 1; rlink[base] = i; rdof[base] = lane; rnrm[base] = -1;
      E.ix[L.rlinkb + base] = -1; E.ix[L.rslot + base] = -1;
      const R bc = glo >= R(0) ? R(1) / h : R(P.beta) / h;
      rbc[base] = bc; rb[base] = bc * glo;
      st3(rd + 3 * base, mk(R(1), R(0), R(0)));
    }
    const int bh = base + (alo ? 1 : 0);
    if (ahi && bh < rcap) {
      rkind[bh] = 2; rlink[bh] = i; rdof[bh] = lane; rnrm[bh] = -1;
      E.ix[L.rlinkb + bh] = -1; E.ix[L.rslot + bh] = -1;
      const R bc = ghi >= R(0) ? R(1) / h : R(P.beta) / h;
      rbc[bh] = bc; rb[bh] = bc * ghi;
      st3(rd + 3 * bh, mk(R(-1), R(0), R(0)));
    }
  }
  int* rlinkb = E.ix + L.rlinkb;
  int* rslot = E.ix + L.rslot;
  for (int s0 = 0; s0 < E.ns; s0 += 64) {
    const int s = s0 + lane;
    bool act = false;
    V3<R> cen = zero3<R>(), x = zero3<R>(), nrm = mk(R(0), R(0), R(1));
    R phi = R(0);
    int i = 0, kb = -1;
    if (s < E.ns) {
      const int* si = M.si + s * SI_COLS;
      const double* sf = M.sf + s * SF_COLS;
      i = si[SI_LINK_A];
      cen = add(ld3<R>(E.at(L.p, i, 3)), mv(E.at(L.Rm, i, 9), ld3<R>(sf + SF_P)));
      const R rad = R(sf[SF_R]);
      if (si[SI_TYPE] == SLOT_SPHERE_BOX) {
        kb = si[SI_LINK_B];
        const R* Rb = E.at(L.Rm, kb, 9);
        const V3<R> bc = add(ld3<R>(E.at(L.p, kb, 3)), mv(Rb, ld3<R>(sf + SF_BOXC)));
        sphere_box(cen, Rb, bc, ld3<R>(sf + SF_HALF), rad, phi, nrm, (R*)nullptr);
      } else {
        phi = cen.z + E.ref.z - rad;
      }
      x = sub(cen, mul(nrm, rad));
      const SV<R> Va = lds6(E.at(L.Vs, i, 6));
      V3<R> u = add(Va.v, cross(Va.w, x));
      if (kb >= 0) {
        const SV<R> Vb = lds6(E.at(L.Vs, kb, 6));
        u = sub(u, add(Vb.v, cross(Vb.w, x)));
      }
      act = phi + h * min_(R(0), dot(nrm, u)) < R(P.mc);
    }
    const unsigned long long m = __ballot(act);
    const int base = nrows + 3 * __popcll(m & lanes_below(lane));
    if (act && base + 2 < rcap) {
      const R bc = phi >= R(0) ? R(1) / h : R(P.beta) / h;
      V3<R> t1, t2, tt;
      tangents(nrm, t1, t2, tt);
      for (int k = 0; k < 3; ++k) {
        const int r = base + k;
        rkind[r] = 3 + k; rlink[r] = i; rdof[r] = -1; rnrm[r] = k == 0 ? -1 : base;
        rlinkb[r] = kb; rslot[r] = s;
        rbc[r] = k == 0 ? bc : R(0);
        rb[r] = k == 0 ? bc * phi : R(0);
        st3(rx + 3 * r, x);
        st3(rcen + 3 * r, cen);
        st3(rd + 3 * r, k == 0 ? nrm : (k == 1 ? t1 : t2));
      }
    }
    nrows += 3 * __popcll(m);
  }
  if (nrows > rcap) return false;
  sync<R>();
  E.phase(9);
  // ---- J rows and responses W = M~^-1 J^T (one row per lane)
  R* J = E.r + L.J;
  R* W = E.r + L.W;
  R Arr = R(0);
  int kind = 0, nrm = -1;
  if (lane < nrows) {
    R* Jr = J + lane * nvp;
    for (int c = 0; c < nv; ++c) Jr[c] = R(0);
    kind = rkind[lane];
    nrm = rnrm[lane];
    const int i = rlink[lane];
    const int* li = E.li(i);
    if (kind <= 2) {
      Jr[li[LI_COL]] = rd[3 * lane];
    } else {
      const V3<R> x = ld3<R>(rx + 3 * lane), d = ld3<R>(rd + 3 * lane);
      if (li[LI_PARENT] >= 0) {
        const SV<R> s = joint_s(E, i);
        Jr[li[LI_COL]] = dot(d, add(s.v, cross(s.w, x)));
      }
      {  // ancestors four at a time, their reads issued together (entries past the last one are not written)
        const int qb = li[LI_ANC_BEGIN], qe = li[LI_ANC_END];
        for (int q0 = qb; q0 < qe; q0 += 4) {
          int col[4];
          R jv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int a = M.anc_link[min(q0 + k, qe - 1)];
            const SV<R> s = joint_s(E, a);
            col[k] = E.li(a)[LI_COL];
            jv[k] = dot(d, add(s.v, cross(s.w, x)));
          }
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (q0 + k < qe) Jr[col[k]] = jv[k];
        }
      }
      const int rt = li[LI_ROOT];
      if (E.li(rt)[LI_JTYPE] == J_FREE) {
        const int c0 = li[LI_ROOTCOL];
        const V3<R> w = cross(sub(x, ld3<R>(E.at(L.c, rt, 3))), d);
        Jr[c0] = d.x; Jr[c0 + 1] = d.y; Jr[c0 + 2] = d.z;
        Jr[c0 + 3] = w.x; Jr[c0 + 4] = w.y; Jr[c0 + 5] = w.z;
      }
      const int kb = E.ix[L.rlinkb + lane];
      if (kb >= 0) {  // body b of a two-body contact enters with the opposite sign
        const int* lb = E.li(kb);
        if (lb[LI_PARENT] >= 0) {
          const SV<R> sv = joint_s(E, kb);
          Jr[lb[LI_COL]] -= dot(d, add(sv.v, cross(sv.w, x)));
        }
        for (int k = lb[LI_ANC_BEGIN]; k < lb[LI_ANC_END]; ++k) {
          const int a = M.anc_link[k];
          const SV<R> sv = joint_s(E, a);
          Jr[E.li(a)[LI_COL]] -= dot(d, add(sv.v, cross(sv.w, x)));
        }
        const int rtb = lb[LI_ROOT];
        if (E.li(rtb)[LI_JTYPE] == J_FREE) {
          const int c0 = lb[LI_ROOTCOL];
          const V3<R> w = cross(sub(x, ld3<R>(E.at(L.c, rtb, 3))), d);
          Jr[c0] -= d.x; Jr[c0 + 1] -= d.y; Jr[c0 + 2] -= d.z;
          Jr[c0 + 3] -= w.x; Jr[c0 + 4] -= w.y; Jr[c0 + 5] -= w.z;
        }
      }
    }
    R* Wr = W + lane * nvp;
    for (int c = 0; c < nv; ++c) Wr[c] = Jr[c];
    chol_solve_row(E, Wr);
    for (int c = 0; c < nv; ++c) Arr += Jr[c] * Wr[c];
  }
  // rows that cannot move are dropped, with the friction rows of a dropped normal
  bool keep = lane < nrows && Arr >= R(kMinRowMass);
  const bool keepn = __shfl(keep, nrm < 0 ? lane : nrm, 64);
  keep = keep && (kind < 4 || keepn);
  const unsigned long long mk_ = __ballot(keep);
  int* rmap = E.ix + L.rmap;
  const int nkeep = __popcll(mk_);
  const int newi = __popcll(mk_ & lanes_below(lane));
  if (keep) rmap[newi] = lane;
  E.R_ = nkeep;
  sync<R>();
  // gather the kept rows' metadata (register copies; tables rewritten below)
  int o = lane < nkeep ? rmap[lane] : 0;
  const int g_kind = __shfl(kind, o, 64), g_link = __shfl(lane < nrows ? rlink[lane] : 0, o, 64);
  const int g_dof = __shfl(lane < nrows ? rdof[lane] : 0, o, 64);
  const int g_linkb = __shfl(lane < nrows ? E.ix[L.rlinkb + lane] : -1, o, 64);
  const int g_slot = __shfl(lane < nrows ? E.ix[L.rslot + lane] : -1, o, 64);
  const int g_nrm_old = __shfl(nrm, o, 64);
  const int g_nrm = __shfl(newi, g_nrm_old < 0 ? 0 : g_nrm_old, 64);
  R g_real[14];
  {
    R mine[14] = {lane < nrows ? rbc[lane] : R(0), lane < nrows ? rb[lane] : R(0), R(1) / (Arr > R(0) ? Arr : R(1))};
    for (int k = 0; k < 3; ++k) {
      mine[3 + k] = lane < nrows ? rx[3 * lane + k] : R(0);
      mine[6 + k] = lane < nrows ? rcen[3 * lane + k] : R(0);
      mine[9 + k] = lane < nrows ? rd[3 * lane + k] : R(0);
    }
    mine[12] = Arr;
    mine[13] = R(0);
#pragma unroll
    for (int k = 0; k < 14; ++k) g_real[k] = __shfl(mine[k], o, 64);
  }
  sync<R>();
  R invA = R(0), bias = R(0);
  if (lane < nkeep) {
    rkind[lane] = g_kind; rlink[lane] = g_link; rdof[lane] = g_dof; rnrm[lane] = g_kind >= 4 ? g_nrm : -1;
    E.ix[L.rlinkb + lane] = g_linkb; E.ix[L.rslot + lane] = g_slot;
    rbc[lane] = g_real[0]; rb[lane] = g_real[1];
    E.r[L.rinvA + lane] = g_real[2];
    for (int k = 0; k < 3; ++k) {
      rx[3 * lane + k] = g_real[3 + k];
      rcen[3 * lane + k] = g_real[6 + k];
      rd[3 * lane + k] = g_real[9 + k];
    }
    invA = g_real[2];
    bias = g_real[1];
  }
  kind = lane < nkeep ? g_kind : 0;
  nrm = lane < nkeep && g_kind >= 4 ? g_nrm : -1;
  sync<R>();
  const int Rn = nkeep;
  E.phase(10);
  // ---- Delassus matrix A = J W^T (symmetric, packed lower), on the matrix cores
  R* A = E.r + L.A;
  const int rcp = L.rcp;
  wave_gemm<R>(
      Rn, Rn, nv, lane, [&](int s, int c) { return J[rmap[s] * nvp + c]; },
      [&](int c, int r) { return W[rmap[r] * nvp + c]; },
      [&](int s, int r, R t) {
        if (r <= s) A[tri(s, r)] = t;
      });
  // ---- Gauss-Seidel with its tape
  R y = R(0), lam = R(0);
  if (lane < Rn) {
    const R* Js = J + rmap[lane] * nvp;
    for (int c = 0; c < nv; ++c) y += Js[c] * vs[c];
  }
  sync<R>();
  R* hlo = E.r + L.hlo;
  R* hres = E.r + L.hres;
  int* hst = E.ix + L.hst;
  const R mu = R(P.mu);
  E.phase(1);
  // every lane evaluates the update of its own row (with the impulse of its normal row, which a friction
  // lane follows through the broadcasts); row r's change is broadcast and applied to every y.  The lane's
  // entry of the next row's column of A is loaded one row ahead.
  const bool fric = kind >= 4;
  const int nrm_own = fric ? nrm : -1;
  const bool own = lane < Rn;
  R lamn = R(0);
  for (int it = 0; it < P.iters; ++it) {
    R a_next = own && Rn > 0 ? A[tri(lane, 0)] : R(0);
    // the lane's own row's tape entries of this sweep, kept in registers by selects and stored once after
    // the sweep (no branch per row)
    R t_lo = R(0), t_res = R(0);
    int t_st = 0;
    for (int r = 0; r < Rn; ++r) {
      const R a_r = a_next;
      if (r + 1 < Rn) a_next = own ? A[tri(lane, r + 1)] : R(0);
      const R res = y + bias;
      const R x = lam - res * invA;
      const R hi = fric ? mu * lamn : R(INFINITY);
      const R lo = fric ? -hi : R(0);
      const int st = x > hi ? 2 : (x < lo ? 1 : 0);
      const R nl = st == 2 ? hi : (st == 1 ? lo : x);
      const R dl = lane_read(nl - lam, r);
      const bool me = lane == r;
      t_lo = me ? lam : t_lo;
      t_res = me ? res : t_res;
      t_st = me ? st : t_st;
      lam = me ? nl : lam;
      lamn += nrm_own == r ? dl : R(0);
      y += a_r * dl;
    }
    if (own) {
      hlo[it * rcp + lane] = t_lo;
      hres[it * rcp + lane] = t_res;
      hst[it * rcp + lane] = t_st;
    }
  }
  if (lane < Rn) E.r[L.rlam + lane] = lam;
  sync<R>();
  E.phase(0);
  R* nu1 = E.r + L.nu1;
  for (int c = lane; c < nv; c += 64) {
    R t = vs[c];
    for (int r = 0; r < Rn; ++r) t += W[rmap[r] * nvp + c] * E.r[L.rlam + r];
    nu1[c] = t;
  }
  sync<R>();
  // ---- semi-implicit integration into sout
  for (int j = lane; j < nd; j += 64) {
    const int c = E.li(E.dof_link(j))[LI_COL];
    sout[13 * na + 2 * j] = q[j] + h * nu1[c];
    sout[13 * na + 2 * j + 1] = nu1[c];
  }
  for (int a = lane; a < na; a += 64) {
    const int* ai = M.ai + a * AI_COLS;
    const R* rs = sin + 13 * a;
    R* ro = sout + 13 * a;
    if (ai[AI_FIXED]) {
      for (int k = 0; k < 7; ++k) ro[k] = rs[k];
      for (int k = 7; k < 13; ++k) ro[k] = R(0);
      continue;
    }
    const R* v = nu1 + ai[AI_COL];
    for (int k = 0; k < 3; ++k) ro[k] = rs[k] + h * v[k];
    R dq[4], q1[4];
    dq_of(mul(mk(v[3], v[4], v[5]), h), dq);
    qmul(dq, rs + 3, q1);
    const R inv = R(1) / sqrt_(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2] + q1[3] * q1[3]);
    for (int k = 0; k < 4; ++k) ro[3 + k] = q1[k] * inv;
    for (int k = 0; k < 6; ++k) ro[7 + k] = v[k];
  }
  sync<R>();
  return true;
}

// ---------------------------------------------------------------- reverse of one substep
// rbar/dbar hold the adjoint of the state after the substep; on return, of the state before it.
// The substep's internals are those left in LDS by fwd_substep(sin, ...).
template <typename R>
__device__ __forceinline__ void rev_substep(Env<R>& E, const R* sin) {
  const AdjArgs& P = *E.P;
  const AdjLds& L = P.L;
  const DevModel& M = P.m;
  const int lane = E.lane, nl = E.nl, nv = E.nv, nd = E.nd, na = E.na;
  const R h = E.h;
  const int nvp = L.nvp, rcp = L.rcp, Rn = E.R_;
  R* rbar = E.r + L.rbar;
  R* dbar = E.r + L.dbar;
  R* nrb = E.r + L.nrb;
  R* nu = E.r + L.nu;
  R* nu1 = E.r + L.nu1;
  R* vs = E.r + L.vs;
  R* qdd = E.r + L.qdd;
  R* nub = E.r + L.nub;
  R* vsb = E.r + L.vsb;
  R* nui = E.r + L.nui;
  R* zz = E.r + L.z;
  R* ww = E.r + L.w;
  R* qb = E.r + L.qb;
  R* ab = E.r + L.ab;
  R* J = E.r + L.J;
  R* W = E.r + L.W;
  R* A = E.r + L.A;
  R* Ab = E.r + L.Ab;
  R* Lm = E.r + L.Lm;
  const int* rmap = E.ix + L.rmap;
  const int* rkind = E.ix + L.rkind;
  const int* rlink = E.ix + L.rlink;
  const int* rdof = E.ix + L.rdof;
  const int* rnrm = E.ix + L.rnrm;
  E.phase(7);
  // ---- clear accumulators (the per-link ones further down: they share the words of the Gauss-Seidel tape)
  for (int c = lane; c < nv; c += 64) nub[c] = R(0);
  for (int k = lane; k < 13 * na; k += 64) nrb[k] = R(0);
  sync<R>();
  // ---- integration reverse
  for (int j = lane; j < nd; j += 64) {
    const int c = E.li(E.dof_link(j))[LI_COL];
    nub[c] = dbar[2 * j + 1] + h * dbar[2 * j];
    qb[j] = dbar[2 * j];
  }
  for (int a = lane; a < na; a += 64) {
    const int* ai = M.ai + a * AI_COLS;
    if (ai[AI_FIXED]) continue;
    const int c = ai[AI_COL];
    const R* rb = rbar + 13 * a;
    for (int k = 0; k < 3; ++k) {
      nrb[13 * a + k] = rb[k];
      nub[c + k] = rb[7 + k] + h * rb[k];
    }
    const V3<R> th = mul(mk(nu1[c + 3], nu1[c + 4], nu1[c + 5]), h);
    R dq[4], q1[4];
    dq_of(th, dq);
    const R* q0 = sin + 13 * a + 3;
    qmul(dq, q0, q1);
    const R n1 = sqrt_(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2] + q1[3] * q1[3]);
    R qo[4], qb1[4];
    R pr = R(0);
    for (int k = 0; k < 4; ++k) {
      qo[k] = rb[3 + k];
      pr += (q1[k] / n1) * qo[k];
    }
    for (int k = 0; k < 4; ++k) qb1[k] = (qo[k] - (q1[k] / n1) * pr) / n1;
    const R dqc[4] = {-dq[0], -dq[1], -dq[2], dq[3]};
    const R q0c[4] = {-q0[0], -q0[1], -q0[2], q0[3]};
    R q0b[4], dqb[4];
    qmul(dqc, qb1, q0b);
    qmul(qb1, q0c, dqb);
    for (int k = 0; k < 4; ++k) nrb[13 * a + 3 + k] = q0b[k];
    const V3<R> thb = dq_adj(th, dqb);
    nub[c + 3] = rb[10] + h * thb.x;
    nub[c + 4] = rb[11] + h * thb.y;
    nub[c + 5] = rb[12] + h * thb.z;
  }
  sync<R>();
  // ---- z = M~^-1 nu_bar;  lambda_bar = J z
  const R zc = chol_solve_lanes(E, lane < nv ? nub[lane] : R(0));
  if (lane < nv) zz[lane] = zc;
  sync<R>();
  const int kind = lane < Rn ? rkind[lane] : 0;
  const int nrm = lane < Rn ? rnrm[lane] : -1;
  const R invA = lane < Rn ? E.r[L.rinvA + lane] : R(0);
  R lamb = R(0), ybar = R(0), bbar = R(0), invAb = R(0);
  if (lane < Rn) {
    const R* Jr = J + rmap[lane] * nvp;
    for (int c = 0; c < nv; ++c) lamb += Jr[c] * zz[c];
  }
  for (int k = lane; k < Rn * (Rn + 1) / 2; k += 64) Ab[k] = R(0);  // S = Abar + Abar^T, packed
  sync<R>();
  // ---- Gauss-Seidel reverse.  q = A ybar is kept up to date (ybar changes in one entry per row
  // update and A is symmetric), so (A^T ybar)_r is read from lane r instead of reduced over the wave.
  const R mu = R(P.mu);
  const R* hlo = E.r + L.hlo;
  const R* hres = E.r + L.hres;
  const R* rlam = E.r + L.rlam;
  const int* hst = E.ix + L.hst;
  R qv = R(0);
  E.phase(2);
  const bool own = lane < Rn;
  for (int it = P.iters - 1; it >= 0; --it) {
    // the lane's own row's tape entries of this sweep, read once; row r's are then taken from lane r
    const int st_own = own ? hst[it * rcp + lane] : 0;
    const R lo_own = own ? hlo[it * rcp + lane] : R(0);
    // lambda after this update: the next sweep's lambda before it, or the final lambda
    const R dl_own = own ? (it + 1 < P.iters ? hlo[(it + 1) * rcp + lane] : rlam[lane]) - lo_own : R(0);
    const R res_own = own ? hres[it * rcp + lane] : R(0);
    R a_next = own && Rn > 0 ? A[tri(lane, Rn - 1)] : R(0);
    for (int r = Rn - 1; r >= 0; --r) {
      const R Asr = a_next;
      if (r > 0) a_next = own ? A[tri(lane, r - 1)] : R(0);
      const int st = lane_read(st_own, r);
      const R dl = lane_read(dl_own, r);
      const R sum = lane_read(qv, r);
      const R g = lane_read(lamb, r) + sum;
      // Abar[s][r] += ybar_s dl enters S[s][r] and S[r][s]: one packed element, twice on the diagonal
      if (own) Ab[tri(lane, r)] += (lane == r ? R(2) : R(1)) * ybar * dl;
      const bool me = lane == r;
      lamb = me ? -sum : lamb;
      if (st == 0) {
        const R dy = -lane_read(invA, r) * g;
        lamb = me ? lamb + g : lamb;
        ybar = me ? ybar + dy : ybar;
        bbar = me ? bbar + dy : bbar;
        invAb = me ? invAb - res_own * g : invAb;
        qv += Asr * dy;
      } else if (lane_read(kind, r) >= 4) {
        const int nr = lane_read(nrm, r);
        if (lane == nr) lamb += (st == 2 ? mu : -mu) * g;
      }
    }
  }
  if (lane < Rn) {
    Ab[tri(lane, lane)] -= R(2) * invAb * invA * invA;
    E.r[L.rybar + lane] = ybar;
    E.r[L.rbbar + lane] = bbar;
  }
  sync<R>();
  E.phase(3);
  // ---- v*_bar = nu_bar + J^T ybar
  for (int c = lane; c < nv; c += 64) {
    R t = nub[c];
    for (int r = 0; r < Rn; ++r) t += J[rmap[r] * nvp + c] * E.r[L.rybar + r];
    vsb[c] = t;
  }
  sync<R>();
  // ---- T_s = sum_r S_sr W_r into the J rows (J is not needed any more)
  wave_gemm<R>(
      Rn, nv, Rn, lane, [&](int s2, int r) { return Ab[tri(s2, r)]; }, [&](int r, int c) { return W[rmap[r] * nvp + c]; },
      [&](int s2, int c, R t) { J[rmap[s2] * nvp + c] = t; });
  // ---- w = M~^-1 (h v*_bar): the adjoint of the generalized forces
  const R wc = chol_solve_lanes(E, lane < nv ? h * vsb[lane] : R(0));
  if (lane < nv) ww[lane] = wc;
  sync<R>();
  // ---- P (dense, into Lm; the factor is not needed any more):
  // P = 1/2 W S W^T + sym(dnu z^T) + sym(qdd w^T), dnu = nu+ - v*
  // (W S W^T = T^T W with T in the J rows)
  wave_gemm<R>(
      nv, nv, Rn, lane, [&](int i, int s2) { return J[rmap[s2] * nvp + i]; }, [&](int s2, int k) { return W[rmap[s2] * nvp + k]; },
      [&](int i, int k, R t) {
        if (k <= i) Lm[lrow(i) + k] = R(0.5) * (t + (nu1[i] - vs[i]) * zz[k] + zz[i] * (nu1[k] - vs[k]) + qdd[i] * ww[k] + ww[i] * qdd[k]);
      });
  sync<R>();
  // ---- Jbar = T + lambda z^T + ybar v*^T
  if (lane < Rn) {
    R* Jr = J + rmap[lane] * nvp;
    const R lr = E.r[L.rlam + lane];
    for (int c = 0; c < nv; ++c) Jr[c] += lr * zz[c] + ybar * vs[c];
  }
  // ---- controls: actuation adjoint, explicit drive terms
  for (int c = lane; c < nv; c += 64) nui[c] = vsb[c];
  sync<R>();
  for (int j = lane; j < nd; j += 64) {
    const int i = E.dof_link(j);
    const int c = E.li(i)[LI_COL];
    const double* lf = E.lf(i);
    const R kp = R(lf[LF_KP]), kd = R(lf[LF_KD]);
    ab[j] += ww[c];
    qb[j] -= kp * ww[c];
    nui[c] -= (h * kp + kd) * ww[c];
  }
  // ---- per-link accumulators, in the words of the Gauss-Seidel tape (read for the last time above)
  sync<R>();
  for (int k = lane; k < 6 * nl; k += 64) {
    E.r[L.wr + k] = R(0);
    E.r[L.sb + k] = R(0);
  }
  for (int k = lane; k < 3 * nl; k += 64) {
    E.r[L.cb + k] = R(0);
    E.r[L.tI + k] = R(0);
  }
  sync<R>();
  E.phase(4);
  // ---- d tr(M P)/dq, weight -1: per column y_k, s_bar and y_bar
  R* colS = E.r + L.colS;
  R* colY = E.r + L.colY;
  R* colYv = E.r + L.colYv;
  for (int k = lane; k < nv; k += 64) {
    const SV<R> sk = col_s(E, k);
    const unsigned long long anc = M.col_anc[k];
    SV<R> y = sz<R>();
    for (int j = 0; j < k; ++j)
      if ((anc >> j) & 1ull) y = sadd(y, smul(col_s(E, j), Lm[lrow(k) + j]));
    const R* Ic = E.at(L.Ic, E.col_link(k), 10);
    const SV<R> Is = comp_mul(Ic, sk), Iy = comp_mul(Ic, y);
    sts6(colS + 6 * k, smul(sadd(Iy, smul(Is, Lm[lrow(k) + k])), R(-2)));
    sts6(colY + 6 * k, smul(Is, R(-2)));
    sts6(colYv + 6 * k, y);
  }
  sync<R>();
  for (int j = lane; j < nv; j += 64) {
    SV<R> a = lds6(colS + 6 * j);
    for (int k = j + 1; k < nv; ++k)
      if ((M.col_anc[k] >> j) & 1ull) a = sadd(a, smul(lds6(colY + 6 * k), Lm[lrow(k) + j]));
    sts6(colS + 6 * j, a);
  }
  sync<R>();
  // per link: inertia adjoints of sum_{k at or above i} -(2 <s_k, I_i y_k> + P_kk <s_k, I_i s_k>),
  // and the column s_bar moved onto the owning link
  for (int i = lane; i < nl; i += 64) {
    const int* li = E.li(i);
    const R m = R(E.lf(i)[LF_MASS]);
    const V3<R> cw = ld3<R>(E.at(L.c, i, 3));
    const R* Iw = E.at(L.Iw, i, 6);
    V3<R> cb = zero3<R>(), tI = zero3<R>();
    const unsigned long long la = M.link_anc[i];
    for (int k = 0; k < nv; ++k) {
      if (!((la >> E.col_link(k)) & 1ull)) continue;
      const SV<R> sk = col_s(E, k);
      bil(m, cw, Iw, sk, lds6(colYv + 6 * k), R(-2), cb, tI);
      bil(m, cw, Iw, sk, sk, -Lm[lrow(k) + k], cb, tI);
    }
    if (li[LI_PARENT] >= 0) {
      acc6(E.at(L.sb, i, 6), lds6(colS + 6 * li[LI_COL]));
    } else if (li[LI_JTYPE] == J_FREE) {
      const int c0 = li[LI_ROOTCOL];
      cb = add(cb, cross(mk(R(1), R(0), R(0)), ld3<R>(colS + 6 * (c0 + 3) + 3)));
      cb = add(cb, cross(mk(R(0), R(1), R(0)), ld3<R>(colS + 6 * (c0 + 4) + 3)));
      cb = add(cb, cross(mk(R(0), R(0), R(1)), ld3<R>(colS + 6 * (c0 + 5) + 3)));
    }
    acc3(E.at(L.cb, i, 3), cb);
    acc3(E.at(L.tI, i, 3), tI);
  }
  sync<R>();
  E.phase(5);
  // ---- C(q, qd) reverse (weight -1, seed w): W_hat, A (RNEA accelerations) outward
  link_vel(E, ww, L.X0);
  {  // per-link terms, independent across links: all links at once
    for (int i = lane; i < E.nl; i += 64) {
      const int* li = E.li(i);
      // X1 still holds the RNEA accelerations of the forward pass; per-link terms:
      const R m = R(E.lf(i)[LF_MASS]);
      const V3<R> cw = ld3<R>(E.at(L.c, i, 3));
      const R* Iw = E.at(L.Iw, i, 6);
      const SV<R> V = lds6(E.at(L.V, i, 6)), Wh = lds6(E.at(L.X0, i, 6)), Ai = lds6(E.at(L.X1, i, 6));
      const SV<R> IV = body_mul(m, cw, Iw, V);
      const SV<R> F = smul(sadd(body_mul(m, cw, Iw, Ai), crf(V, IV)), R(-1));
      const SV<R> Ab_ = smul(body_mul(m, cw, Iw, Wh), R(-1));
      V3<R> cb = zero3<R>(), tI = zero3<R>();
      bil(m, cw, Iw, Wh, Ai, R(-1), cb, tI);
      const SV<R> Y = smul(crm(V, Wh), R(-1));
      bil(m, cw, Iw, Y, V, R(-1), cb, tI);
      const SV<R> Vb = smul(sadd(smul(crf(Wh, IV), R(-1)), body_mul(m, cw, Iw, Y)), R(-1));
      acc3(E.at(L.cb, i, 3), cb);
      acc3(E.at(L.tI, i, 3), tI);
      sts6(E.at(L.X2, i, 6), F);
      sts6(E.at(L.X3, i, 6), Ab_);
      sts6(E.at(L.X0, i, 6), Vb);
      (void)li;
    }
  }
  sync<R>();
  // inward: subtree sums of F, Abar, Vbar (Vbar of a parent also receives qd crf(s, Abar) of each child)
  for (int lev = E.nlev - 1; lev >= 0; --lev) {
    const int b = E.lev_begin(lev), e = E.lev_begin(lev + 1);
    for (int t = b + lane; t < e; t += 64) {
      const int i = E.lev_link(t);
      const int* li = E.li(i);
      SV<R> F = lds6(E.at(L.X2, i, 6)), Ab_ = lds6(E.at(L.X3, i, 6)), Vb = lds6(E.at(L.X0, i, 6));
      for (int k = li[LI_CHILD_BEGIN]; k < li[LI_CHILD_END]; ++k) {
        const int ch = E.child(k);
        const SV<R> Ach = lds6(E.at(L.X3, ch, 6));
        F = sadd(F, lds6(E.at(L.X2, ch, 6)));
        Ab_ = sadd(Ab_, Ach);
        Vb = sadd(Vb, sadd(lds6(E.at(L.X0, ch, 6)), smul(crf(joint_s(E, ch), Ach), nu[E.li(ch)[LI_COL]])));
      }
      sts6(E.at(L.X2, i, 6), F);
      sts6(E.at(L.X3, i, 6), Ab_);
      sts6(E.at(L.X0, i, 6), Vb);
      if (li[LI_PARENT] < 0 && li[LI_JTYPE] == J_FREE) {
        const int c = li[LI_ROOTCOL];
        const V3<R> v = mk(nu[c], nu[c + 1], nu[c + 2]), w = mk(nu[c + 3], nu[c + 4], nu[c + 5]);
        const V3<R> wwv = mk(ww[c + 3], ww[c + 4], ww[c + 5]);
        const V3<R> c0 = ld3<R>(E.at(L.c, i, 3));
        V3<R> cb = add(cross(wwv, F.v), cross(w, Vb.v));
        acc3(E.at(L.cb, i, 3), cb);
        const V3<R> nv_ = add(cross(w, Ab_.v), Vb.v);
        const V3<R> nw_ = add(add(cross(Ab_.v, v), Vb.w), cross(Vb.v, c0));
        nui[c] += nv_.x; nui[c + 1] += nv_.y; nui[c + 2] += nv_.z;
        nui[c + 3] += nw_.x; nui[c + 4] += nw_.y; nui[c + 5] += nw_.z;
      }
    }
    sync<R>();
  }
  // joint terms of every non-root link at once from its summed F, Abar, Vbar
  for (int i = lane; i < E.nl; i += 64) {
    const int* li = E.li(i);
    if (li[LI_PARENT] < 0) continue;
    const SV<R> F = lds6(E.at(L.X2, i, 6)), Ab_ = lds6(E.at(L.X3, i, 6)), Vb = lds6(E.at(L.X0, i, 6));
    const int c = li[LI_COL];
    const SV<R> s = joint_s(E, i), Vp = lds6(E.at(L.V, li[LI_PARENT], 6));
    const SV<R> sb = sadd(sadd(smul(F, ww[c]), smul(crf(Vp, Ab_), -nu[c])), smul(Vb, nu[c]));
    acc6(E.at(L.sb, i, 6), sb);
    nui[c] += sdot(Ab_, crm(Vp, s)) + sdot(s, Vb);
  }
  sync<R>();
  E.phase(6);
  // ---- constraint rows: per row, the adjoints of its contact point (x) and direction (d) from the
  // velocities Jbar_r induces on its bodies; limit rows: the bias adjoint of the joint position
  R* rxb = E.r + L.rxb;
  R* rdb = E.r + L.rdb;
  R* rqb = E.r + L.rqb;
  const int* rlinkb = E.ix + L.rlinkb;
  auto path_vel = [&](int i, const R* Jr) {
    const int* li = E.li(i);
    SV<R> Vt = sz<R>();
    if (li[LI_PARENT] >= 0) Vt = smul(joint_s(E, i), Jr[li[LI_COL]]);
    // ancestors four at a time, their reads issued together (entries past the last one read the last one
    // again and add zero)
    const int qb = li[LI_ANC_BEGIN], qe = li[LI_ANC_END];
    for (int q0 = qb; q0 < qe; q0 += 4) {
      SV<R> sv[4];
      R jc[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int a = M.anc_link[min(q0 + k, qe - 1)];
        sv[k] = joint_s(E, a);
        const R j = Jr[E.li(a)[LI_COL]];
        jc[k] = q0 + k < qe ? j : R(0);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) Vt = sadd(Vt, smul(sv[k], jc[k]));
    }
    const int rt = li[LI_ROOT];
    if (E.li(rt)[LI_JTYPE] == J_FREE) Vt = sadd(Vt, root_vel(ld3<R>(E.at(L.c, rt, 3)), Jr + li[LI_ROOTCOL]));
    return Vt;
  };
  if (lane < Rn) {
    const R* Jr = J + rmap[lane] * nvp;
    const R bc = E.r[L.rbc + lane];
    if (kind >= 3) {
      const V3<R> x = ld3<R>(E.r + L.rx + 3 * lane), d = ld3<R>(E.r + L.rd + 3 * lane);
      const SV<R> Va = path_vel(rlink[lane], Jr);
      V3<R> u = add(Va.v, cross(Va.w, x)), wd = Va.w;
      const int kb = rlinkb[lane];
      if (kb >= 0) {
        const SV<R> Vb = path_vel(kb, Jr);
        u = sub(u, add(Vb.v, cross(Vb.w, x)));
        wd = sub(wd, Vb.w);
      }
      st3(rxb + 3 * lane, cross(d, wd));
      st3(rdb + 3 * lane, u);
      rqb[lane] = R(0);
    } else {
      st3(rxb + 3 * lane, zero3<R>());
      st3(rdb + 3 * lane, zero3<R>());
      rqb[lane] = bbar * bc * E.r[L.rd + 3 * lane];
    }
  }
  sync<R>();
  // per contact (the lane of its normal row): x = c - rad n, d = n, t1(n), t2(n), bias from phi; the
  // sphere centre c moves with body a; for a box partner, phi and n move with c relative to the box
  // (ub = phib n + G^T nb) and n turns with the box: body a gets (c x ca, ca) with ca = cb + ub, body b
  // gets (n x nb - c x ub, -ub)
  R* rwa = E.r + L.rwa;
  R* rwb = E.r + L.rwb;
  if (lane < Rn && kind == 3) {
    const int sl = E.ix[L.rslot + lane];
    const double* sf = M.sf + sl * SF_COLS;
    const R rad = R(sf[SF_R]);
    const V3<R> c = ld3<R>(E.r + L.rcen + 3 * lane), n = ld3<R>(E.r + L.rd + 3 * lane);
    V3<R> cb = ld3<R>(rxb + 3 * lane), t1b = zero3<R>(), t2b = zero3<R>();
    V3<R> nb = ld3<R>(rdb + 3 * lane);
    // a contact's friction rows are generated right after its normal row and compaction keeps the order,
    // so only the next two rows can refer to this one
    for (int r = lane + 1; r <= lane + 2 && r < Rn; ++r) {
      if (rnrm[r] != lane) continue;
      cb = add(cb, ld3<R>(rxb + 3 * r));
      if (rkind[r] == 4) t1b = add(t1b, ld3<R>(rdb + 3 * r));
      else t2b = add(t2b, ld3<R>(rdb + 3 * r));
    }
    nb = sub(nb, mul(cb, rad));
    const R phib = bbar * E.r[L.rbc + lane];
    const int kb = rlinkb[lane];
    SV<R> wa, wb = sz<R>();
    if (kb < 0) {
      cb.z += phib;
      wa = {cross(c, cb), cb};
    } else {
      nb = add(nb, tangents_adj(n, t1b, t2b));
      const R* Rb = E.at(L.Rm, kb, 9);
      const V3<R> bcen = add(ld3<R>(E.at(L.p, kb, 3)), mv(Rb, ld3<R>(sf + SF_BOXC)));
      R phi_, G[9];
      V3<R> n_;
      sphere_box(c, Rb, bcen, ld3<R>(sf + SF_HALF), rad, phi_, n_, G);
      const V3<R> ub = add(mul(n, phib), mk(G[0] * nb.x + G[3] * nb.y + G[6] * nb.z, G[1] * nb.x + G[4] * nb.y + G[7] * nb.z,
                                            G[2] * nb.x + G[5] * nb.y + G[8] * nb.z));
      const V3<R> ca = add(cb, ub);
      wa = {cross(c, ca), ca};
      wb = {sub(cross(n, nb), cross(c, ub)), mul(ub, R(-1))};
    }
    sts6(rwa + 6 * lane, wa);
    sts6(rwb + 6 * lane, wb);
  }
  sync<R>();
  for (int i = lane; i < nl; i += 64) {
    const int* li = E.li(i);
    SV<R> sb = sz<R>();
    V3<R> cb = zero3<R>();
    SV<R> xw = sz<R>();
    for (int r = 0; r < Rn; ++r) {
      if (rkind[r] < 3) continue;
      const int la = rlink[r], lb = rlinkb[r];
      const R* Jr = J + rmap[r] * nvp;
      const V3<R> x = ld3<R>(E.r + L.rx + 3 * r), d = ld3<R>(E.r + L.rd + 3 * r);
      for (int side = 0; side < 2; ++side) {
        const int lk = side == 0 ? la : lb;
        if (lk < 0) continue;
        const R sgn = side == 0 ? R(1) : R(-1);
        if (li[LI_PARENT] >= 0) {
          if ((M.link_anc[lk] >> i) & 1ull) sb = sadd(sb, smul(SV<R>{cross(x, d), d}, sgn * Jr[li[LI_COL]]));
        } else if (li[LI_JTYPE] == J_FREE && E.li(lk)[LI_ROOT] == i) {
          cb = add(cb, mul(cross(ld3<R>(Jr + li[LI_ROOTCOL] + 3), d), sgn));
        }
      }
      if (rkind[r] == 3) {
        if (la == i) xw = sadd(xw, lds6(rwa + 6 * r));
        if (lb == i) xw = sadd(xw, lds6(rwb + 6 * r));
      }
    }
    acc6(E.at(L.sb, i, 6), sb);
    acc3(E.at(L.cb, i, 3), cb);
    acc6(E.at(L.wr, i, 6), xw);
  }
  for (int j = lane; j < nd; j += 64)
    for (int r = 0; r < Rn; ++r)
      if (rkind[r] <= 2 && rdof[r] == j) qb[j] += rqb[r];
  sync<R>();
  // ---- world adjoints -> one wrench per link
  for (int i = lane; i < nl; i += 64) {
    const int* li = E.li(i);
    const V3<R> cw = ld3<R>(E.at(L.c, i, 3)), cb = ld3<R>(E.at(L.cb, i, 3));
    SV<R> Wr = sadd(lds6(E.at(L.wr, i, 6)), SV<R>{add(cross(cw, cb), ld3<R>(E.at(L.tI, i, 3))), cb});
    if (li[LI_PARENT] >= 0) {
      const SV<R> sb = lds6(E.at(L.sb, i, 6));
      const V3<R> ax = ld3<R>(E.at(L.ax, i, 3)), o = ld3<R>(E.at(L.p, i, 3));
      if (li[LI_JTYPE] == J_REV) {
        const V3<R> axb = add(sb.w, cross(sb.v, o));
        const V3<R> ob = cross(ax, sb.v);
        Wr = sadd(Wr, SV<R>{add(cross(ax, axb), cross(o, ob)), ob});
      } else {
        Wr.w = add(Wr.w, cross(ax, sb.v));
      }
    }
    sts6(E.at(L.wr, i, 6), Wr);
  }
  sync<R>();
  // subtree sums (inward), position adjoints
  for (int lev = E.nlev - 1; lev >= 0; --lev) {
    const int b = E.lev_begin(lev), e = E.lev_begin(lev + 1);
    for (int t = b + lane; t < e; t += 64) {
      const int i = E.lev_link(t);
      const int* li = E.li(i);
      SV<R> Wc = lds6(E.at(L.wr, i, 6));
      for (int k = li[LI_CHILD_BEGIN]; k < li[LI_CHILD_END]; ++k) Wc = sadd(Wc, lds6(E.at(L.wr, E.child(k), 6)));
      sts6(E.at(L.wr, i, 6), Wc);
      if (li[LI_PARENT] < 0 && li[LI_JTYPE] == J_FREE) {
        int a = 0;
        while (M.ai[a * AI_COLS + AI_ROOT] != i) ++a;
        const V3<R> p0 = ld3<R>(E.at(L.p, i, 3));
        acc3(nrb + 13 * a, Wc.v);
        const V3<R> dth = sub(Wc.w, cross(p0, Wc.v));
        const R* q = sin + 13 * a + 3;
        const R nq = sqrt_(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const R t4[4] = {dth.x, dth.y, dth.z, R(0)};
        const R qh[4] = {q[0] / nq, q[1] / nq, q[2] / nq, q[3] / nq};
        R o4[4];
        qmul(t4, qh, o4);
        for (int k = 0; k < 4; ++k) nrb[13 * a + 3 + k] += R(2) * o4[k] / nq;
      }
    }
    sync<R>();
  }
  for (int i = lane; i < E.nl; i += 64) {  // joint-position adjoints of every non-root link at once
    const int* li = E.li(i);
    if (li[LI_PARENT] >= 0) qb[li[LI_DOF]] += sdot(joint_s(E, i), lds6(E.at(L.wr, i, 6)));
  }
  sync<R>();
  E.phase(7);
  // ---- adjoint of the substep's start state
  for (int j = lane; j < nd; j += 64) {
    dbar[2 * j] = qb[j];
    dbar[2 * j + 1] = nui[E.li(E.dof_link(j))[LI_COL]];
  }
  for (int a = lane; a < na; a += 64) {
    const int* ai = M.ai + a * AI_COLS;
    R* rb = rbar + 13 * a;
    if (ai[AI_FIXED]) {
      for (int k = 0; k < 13; ++k) rb[k] = R(0);
      continue;
    }
    const int c = ai[AI_COL];
    for (int k = 0; k < 7; ++k) rb[k] = nrb[13 * a + k];
    for (int k = 0; k < 6; ++k) rb[7 + k] = nui[c + k];
  }
  sync<R>();
}

// the adjoint of entry ei of the launch's env list, by one 64-lane workgroup
template <typename R>
__device__ __forceinline__ void adjoint_env(const AdjArgs& P, int ei) {
  extern __shared__ double g_adj_lds[];
  const AdjLds& L = P.L;
  Env<R> E;
  E.P = &P;
  E.r = reinterpret_cast<R*>(g_adj_lds);
  E.ix = reinterpret_cast<int*>(E.r + L.n_real);
  E.lane = threadIdx.x;
  E.nl = P.m.n_links;
  E.nv = P.m.n_v;
  E.nd = P.m.n_dof;
  E.na = P.m.n_actors;
  E.ns = P.m.n_slots;
  E.nlev = P.m.n_levels;
  E.rc = L.rows_cap;
  if (Env<R>::kStaged) {  // stage the model's integer tables (every lane copies; the sync below orders them)
    const DevModel& G = P.m;
    int* ix = E.ix;
    for (int k = E.lane; k < G.n_links * LI_COLS; k += 64) ix[L.t_li + k] = G.li[k];
    for (int k = E.lane; k <= G.n_levels; k += 64) ix[L.t_lev + k] = G.level_begin[k];
    for (int k = E.lane; k < G.n_links; k += 64) ix[L.t_links + k] = G.level_links[k];
    for (int k = E.lane; k < G.n_links - G.n_actors; k += 64) ix[L.t_child + k] = G.children[k];
    for (int k = E.lane; k < G.n_v; k += 64) ix[L.t_col + k] = G.col_link[k];
    for (int k = E.lane; k < G.n_dof; k += 64) ix[L.t_dof + k] = G.dof_link[k];
  }
  const int env = P.env_list[ei];
  if (P.skip_flags && P.skip_flags[env] != 0) return;  // another launch runs this env
  E.abase = P.env_actor_base[env];
  E.dbase = P.env_dof_base[env];
  E.h = R(P.h);
  E.g = mk(R(P.gx), R(P.gy), R(P.gz));
  if (P.cycles && E.lane == 0) {
    for (int k = 0; k < kAdjPhases; ++k) g_adj_clock[k] = 0;
    g_adj_clock[kAdjPhases] = -1;
  }
  const int lane = E.lane, na = E.na, nd = E.nd, sw = L.state_words, S = P.substeps;
  R* st = E.r + L.st;
  // step start state and the adjoint of the step's end state
  for (int k = lane; k < 13 * na; k += 64) {
    st[k] = R(P.root_state[(long long)E.abase * 13 + k]);
    E.r[L.rbar + k] = R(P.root_adj[(long long)E.abase * 13 + k]);
  }
  for (int k = lane; k < 2 * nd; k += 64) {
    st[13 * na + k] = R(P.dof_state[(long long)E.dbase * 2 + k]);
    E.r[L.dbar + k] = R(P.dof_adj[(long long)E.dbase * 2 + k]);
  }
  for (int j = lane; j < nd; j += 64) E.r[L.ab + j] = R(0);
  sync<R>();
  E.ref = mk(st[0], st[1], st[2]);
  bool ok = true;
  if (P.mid_root) {  // substep start states handed over by the forward step
    for (int s = 1; s < S; ++s) {
      const double* mr = P.mid_root + (long long)(s - 1) * P.mid_block + (long long)E.abase * 13;
      const double* md = P.mid_dof + (long long)(s - 1) * P.mid_block + (long long)E.dbase * 2;
      for (int k = lane; k < 13 * na; k += 64) st[s * sw + k] = R(mr[k]);
      for (int k = lane; k < 2 * nd; k += 64) st[s * sw + 13 * na + k] = R(md[k]);
    }
    sync<R>();
  } else {
    for (int s = 0; s + 1 < S && ok; ++s) ok = fwd_substep(E, st + s * sw, st + (s + 1) * sw);
  }
  for (int s = S - 1; s >= 0 && ok; --s) {
    ok = fwd_substep(E, st + s * sw, st + S * sw);
    if (ok) rev_substep(E, st + s * sw);
  }
  if (!ok && P.retry) {  // more rows than this layout holds: hand the environment to the larger layout
    if (lane == 0) P.retry[atomicAdd(P.retry_count, 1)] = env;
    return;
  }
  for (int k = lane; k < 13 * na; k += 64) P.root_adj[(long long)E.abase * 13 + k] = ok ? float(E.r[L.rbar + k]) : 0.0f;
  for (int k = lane; k < 2 * nd; k += 64) P.dof_adj[(long long)E.dbase * 2 + k] = ok ? float(E.r[L.dbar + k]) : 0.0f;
  for (int j = lane; j < nd; j += 64) P.act_adj[E.dbase + j] = ok ? float(E.r[L.ab + j]) : 0.0f;
  if (P.status && lane == 0 && (!ok || !P.status_sticky)) P.status[env] = ok ? 0 : 1;
  E.phase(-1);
  if (P.cycles && lane == 0)
    for (int k = 0; k < kAdjPhases; ++k) P.cycles[(long long)env * kAdjPhases + k] = g_adj_clock[k];
}

// Register budget: FP32 forms at two wavefronts per SIMD (<= 256 registers: LDS admits six workgroups per
// CU with the humanoid's small layout); FP64 forms at one (their LDS admits three workgroups per CU anyway)
template <typename R>
constexpr int kAdjWavesPerEU = sizeof(R) == 4 ? 2 : 1;

// one env per workgroup
template <typename R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kAdjWavesPerEU<R>))) void adjoint_kernel(AdjArgs P, int n_envs) {
  const int ei = blockIdx.x;
  if (ei >= n_envs || (P.list_count && ei >= *P.list_count)) return;
  adjoint_env<R>(P, ei);
}
// fewer workgroups than list entries, each striding over the device list (the flagged-env pass); kept apart
// from adjoint_kernel because the loop costs registers (a few spilled in the FP32 form)
template <typename R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kAdjWavesPerEU<R>))) void adjoint_list_kernel(AdjArgs P, int n_envs) {
  // The flagged envs (more rows, the larger layout) share their CUs with the first pass and would otherwise
  // finish last and set the step's time: their wavefronts take the highest issue priority on their SIMD.
  __builtin_amdgcn_s_setprio(3);
  for (int ei = blockIdx.x; ei < n_envs; ei += gridDim.x) {
    if (ei >= *P.list_count) return;
    adjoint_env<R>(P, ei);
    __syncthreads();  // the next entry reuses the LDS
  }
}

__global__ void zero_count_kernel(int* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// list[0] = number of envs of env_list[0, n) whose flag is set, list[1 ...] = those envs (any order)
__global__ void compact_flags_kernel(const int* env_list, int n, const int* flags, int* list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int env = env_list[i];
  if (flags[env] != 0) list[1 + atomicAdd(list, 1)] = env;
}

template <typename R>
hipError_t launch_adj(const AdjArgs& a, int n_envs, int grid, hipStream_t stream) {
  const size_t lds = (size_t)a.L.n_real * sizeof(R) + (size_t)a.L.n_int * sizeof(int);
  if (grid < n_envs) hipLaunchKernelGGL(adjoint_list_kernel<R>, dim3(grid), dim3(64), lds, stream, a, n_envs);
  else hipLaunchKernelGGL(adjoint_kernel<R>, dim3(grid), dim3(64), lds, stream, a, n_envs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs& a, int n_envs, int fp64, hipStream_t stream, int grid) {
  if (n_envs <= 0) return hipSuccess;
  grid = (grid > 0 && grid < n_envs) ? grid : n_envs;
  if (grid < n_envs && !a.list_count) return hipErrorInvalidValue;
  return fp64 ? launch_adj<double>(a, n_envs, grid, stream) : launch_adj<float>(a, n_envs, grid, stream);
}

hipError_t launch_compact_flags(const int* env_list, int n, const int* flags, int* list, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_flags_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, env_list, n, flags, list);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t launch_fill_int(int* p, int n, int value, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, value);
  return hipGetLastError();
}

hipError_t launch_zero_count(int* c, hipStream_t stream) {
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, stream, c);
  return hipGetLastError();
}

hipError_t set_adjoint_lds_limit(int fp64, size_t bytes) {
  const void* f = fp64 ? (const void*)adjoint_kernel<double> : (const void*)adjoint_kernel<float>;
  const void* g = fp64 ? (const void*)adjoint_list_kernel<double> : (const void*)adjoint_list_kernel<float>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

}  // namespace ags
