// Batched articulated-physics step for gfx950: one wavefront (64 lanes) per environment.
//
// Per substep h = dt / substeps, for every environment (Section 3: reduced-coordinate
// articulations; Table 3: sim parameters; Table 4: 2 substeps per control step):
//   controls -> joint forces (actuation + implicit PD drive)
//   forward sweep: kinematics, link inertias, velocities, velocity-product and bias forces
//   articulated-body algorithm (Featherstone 2008, ch. 7): inward sweep, root solve, outward sweep
//   narrow phase (sphere/capsule/box vs plane, sphere/capsule vs box) with speculative activation
//   constraint rows: joint limits and contacts (normal + 2 friction directions)
//   row responses W_r = M~^-1 J_r^T by articulated unit-load sweeps reusing the ABA factors
//   fixed-sweep projected Gauss-Seidel on the joint velocities
//   semi-implicit integration and output accumulation
//
// Frames: every spatial quantity of link i is expressed with world-aligned axes about the link's
// own joint origin o_i (a free root: its centre of mass), positions relative to the first actor's
// root.  Moving a quantity between links is a pure translation, so the inward sweep needs no
// rotations and every lever arm stays at the size of one link.
//
// The kernel is a template over the compute type R.  R = float is the FP32 path; R = double keeps
// the same FP32 tensors but computes in FP64, which gfx950's vector units issue at the FP32
// (unpacked) rate; joint-space conditioning of the humanoid (cond(M~) ~ 2e3) puts FP32 results about
// 1e-4 away from the exact ones.
#include "ags_internal.h"

namespace ags {
namespace {

// ---------------------------------------------------------------- scalar helpers
__device__ __forceinline__ float rsqrt_(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float min_(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double min_(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float max_(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double max_(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float abs_(float a) { return fabsf(a); }
__device__ __forceinline__ double abs_(double a) { return fabs(a); }
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
template <typename R, typename P>
__device__ __forceinline__ V3<R> ld3(const P& p) {
  return {R(p[0]), R(p[1]), R(p[2])};
}
template <typename R, typename P>
__device__ __forceinline__ void st3(const P& p, V3<R> v) {
  p[0] = v.x;
  p[1] = v.y;
  p[2] = v.z;
}
template <typename R>
__device__ __forceinline__ void st3(R* p, V3<R> v) {
  p[0] = v.x;
  p[1] = v.y;
  p[2] = v.z;
}
// 3x3 row-major helpers
template <typename R, typename P>
__device__ __forceinline__ V3<R> mv(const P& M, V3<R> v) {
  return {M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
          M[6] * v.x + M[7] * v.y + M[8] * v.z};
}
template <typename R, typename P>
__device__ __forceinline__ V3<R> mtv(const P& M, V3<R> v) {
  return {M[0] * v.x + M[3] * v.y + M[6] * v.z, M[1] * v.x + M[4] * v.y + M[7] * v.z,
          M[2] * v.x + M[5] * v.y + M[8] * v.z};
}
// symmetric 3x3 stored xx yy zz xy xz yz
template <typename R>
__device__ __forceinline__ V3<R> symv(const R* S, V3<R> v) {
  return {S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
          S[4] * v.x + S[5] * v.y + S[2] * v.z};
}
template <typename PA, typename PB, typename R>
__device__ __forceinline__ void mm3(const PA& A, const PB& B, R* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// ---------------------------------------------------------------- spatial inertia (21 words)
// A (sym 3x3, angular block), B (3x3 row-major coupling), M (sym 3x3): I [w; v] = [A w + B v; B^T w + M v]
template <typename R>
struct SI {
  R A[6], B[9], M[6];
};
template <typename R, typename P>
__device__ __forceinline__ void si_load(SI<R>& I, const P& p) {
#pragma unroll
  for (int k = 0; k < 6; ++k) I.A[k] = p[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) I.B[k] = p[6 + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) I.M[k] = p[15 + k];
}
template <typename R, typename P>
__device__ __forceinline__ void si_store(const SI<R>& I, const P& p) {
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = I.A[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) p[6 + k] = I.B[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[15 + k] = I.M[k];
}
template <typename R, typename P>
__device__ __forceinline__ void si_addload(SI<R>& I, const P& p) {
#pragma unroll
  for (int k = 0; k < 6; ++k) I.A[k] += p[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) I.B[k] += p[6 + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) I.M[k] += p[15 + k];
}
template <typename R>
__device__ __forceinline__ void si_mul(const SI<R>& I, V3<R> w, V3<R> v, V3<R>& ra, V3<R>& rl) {
  ra = add(symv(I.A, w), mv(I.B, v));
  rl = add(mtv(I.B, w), symv(I.M, v));
}
template <typename R>
__device__ __forceinline__ R si_at(const SI<R>& I, int r, int c) {
  const int sidx[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
  if (r < 3 && c < 3) return I.A[sidx[3 * r + c]];
  if (r < 3) return I.B[3 * r + (c - 3)];
  if (c < 3) return I.B[3 * c + (r - 3)];
  return I.M[sidx[3 * (r - 3) + (c - 3)]];
}
// stored index of entry (m, n) of a spatial inertia [A B; B^T M] in the 21-word layout
__device__ __forceinline__ int si_index(int m, int n) {
  const int lo = min(m, n), hi = max(m, n);
  if (hi < 3) return lo == hi ? lo : lo + hi + 2;              // A: xx yy zz xy xz yz
  if (lo >= 3) return lo == hi ? 12 + lo : 15 + lo + hi - 4;  // M: xx yy zz xy xz yz
  return 6 + 3 * lo + (hi - 3);                                // B row-major (B^T entries read B)
}
// Move an inertia from point Q to point P = Q - r (translation only): I_P = X^T I_Q X with
// X = [1 0; -r^ 1].  Then M' = M, B' = B + r^ M, A' = A - B r^ + r^ B'^T.
template <typename R>
__device__ __forceinline__ void si_shift(SI<R>& I, V3<R> r) {
  const int sidx[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
  R Mf[9], Bn[9], Af[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Mf[k] = I.M[sidx[k]];
#pragma unroll
  for (int j = 0; j < 3; ++j) {  // columns of B': B[:, j] + r x M[:, j]
    V3<R> x = cross(r, mk(Mf[j], Mf[3 + j], Mf[6 + j]));
    Bn[j] = I.B[j] + x.x;
    Bn[3 + j] = I.B[3 + j] + x.y;
    Bn[6 + j] = I.B[6 + j] + x.z;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // rows of -B r^: -(B row i) x r
    V3<R> q = cross(mk(I.B[3 * i], I.B[3 * i + 1], I.B[3 * i + 2]), r);
    Af[3 * i + 0] = -q.x;
    Af[3 * i + 1] = -q.y;
    Af[3 * i + 2] = -q.z;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // columns of r^ B'^T: r x (B' row i)
    V3<R> pc = cross(r, mk(Bn[3 * i], Bn[3 * i + 1], Bn[3 * i + 2]));
    Af[0 + i] += pc.x;
    Af[3 + i] += pc.y;
    Af[6 + i] += pc.z;
  }
  const R half = R(0.5);
  I.A[0] += Af[0];
  I.A[1] += Af[4];
  I.A[2] += Af[8];
  I.A[3] += half * (Af[1] + Af[3]);
  I.A[4] += half * (Af[2] + Af[6]);
  I.A[5] += half * (Af[5] + Af[7]);
#pragma unroll
  for (int k = 0; k < 9; ++k) I.B[k] = Bn[k];
}

template <typename R>
__device__ __forceinline__ R wave_sum(R x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}
__device__ __forceinline__ unsigned long long lanes_below(int t) { return (1ull << t) - 1ull; }
// ballot of one team (TEAM consecutive lanes starting at tm * TEAM), as a mask over its own lanes
template <int TEAM>
__device__ __forceinline__ unsigned long long team_ballot(int tm, int pred) {
  const unsigned long long m = __ballot(pred);
  if (TEAM == 64) return m;
  return (m >> (tm * TEAM)) & ((1ull << TEAM) - 1ull);
}
// sum over the lanes of one team (butterfly within aligned groups of TEAM lanes)
template <int TEAM, typename R>
__device__ __forceinline__ R team_sum(R x) {
#pragma unroll
  for (int m = TEAM / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}
// value of x in lane l (l uniform across the wave)
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
// value of x in lane r of this lane's team (r uniform); one readlane per team, then a select
template <int TEAM, typename T>
__device__ __forceinline__ T team_read(int tm, T x, int r) {
  if (TEAM == 64) return lane_read(x, r);
  T v = lane_read(x, r);
#pragma unroll
  for (int q = 1; q < 64 / TEAM; ++q) {
    const T w = lane_read(x, q * TEAM + r);
    v = tm == q ? w : v;
  }
  return v;
}
// x in the lane of this team given by the team-local index held in idx at team lane r
template <int TEAM, typename T>
__device__ __forceinline__ T team_read_at(T x, int idx, int r, int tm) {
  if (TEAM == 64) return lane_read(x, lane_read(idx, r));
  T v = lane_read(x, lane_read(idx, r));
#pragma unroll
  for (int q = 1; q < 64 / TEAM; ++q) {
    const T w = lane_read(x, q * TEAM + lane_read(idx, q * TEAM + r));
    v = tm == q ? w : v;
  }
  return v;
}

// Cholesky of a 6x6 SPD matrix (packed lower, index i(i+1)/2 + j) and the reciprocal diagonal
template <typename R, typename P>
__device__ __forceinline__ void chol6(const SI<R>& K, const P& L, const P& dinv) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    R d = si_at(K, j, j);
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
    d = sqrt_(max_(d, R(1e-30)));
    L[j * (j + 1) / 2 + j] = d;
    R inv = R(1) / d;
    dinv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      R s = si_at(K, i, j);
#pragma unroll
      for (int k = 0; k < j; ++k) s -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = s * inv;
    }
  }
}
template <typename R, typename P>
__device__ __forceinline__ void chol6_solve(const P& L, const P& dinv, R* x) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R s = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= L[i * (i + 1) / 2 + k] * x[k];
    x[i] = s * dinv[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    R s = x[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s -= L[k * (k + 1) / 2 + i] * x[k];
    x[i] = s * dinv[i];
  }
}

// rotation of angle q about unit axis a (Rodrigues), row-major
template <typename R>
__device__ __forceinline__ void axis_angle(V3<R> a, R q, R* M) {
  R s, c;
  sincos_(q, &s, &c);
  R t = R(1) - c;
  M[0] = c + t * a.x * a.x;
  M[1] = t * a.x * a.y - s * a.z;
  M[2] = t * a.x * a.z + s * a.y;
  M[3] = t * a.x * a.y + s * a.z;
  M[4] = c + t * a.y * a.y;
  M[5] = t * a.y * a.z - s * a.x;
  M[6] = t * a.x * a.z - s * a.y;
  M[7] = t * a.y * a.z + s * a.x;
  M[8] = c + t * a.z * a.z;
}

// tangent basis of a contact normal: t1 = normalised projection of the world axis least aligned with n
// (lowest index on ties), t2 = n x t1
template <typename R>
__device__ __forceinline__ void tangents(V3<R> n, V3<R>& t1, V3<R>& t2) {
  R ax = abs_(n.x), ay = abs_(n.y), az = abs_(n.z);
  int k = 0;
  R best = ax;
  if (ay < best) {
    best = ay;
    k = 1;
  }
  if (az < best) k = 2;
  V3<R> e = k == 0 ? mk(R(1), R(0), R(0)) : (k == 1 ? mk(R(0), R(1), R(0)) : mk(R(0), R(0), R(1)));
  V3<R> t = sub(e, mul(n, dot(n, e)));
  t1 = mul(t, rsqrt_(dot(t, t)));
  t2 = cross(n, t1);
}

// LDS array of one environment.  The EPW environments of a wavefront are interleaved element by
// element (element k of team tm sits at base[k * EPW + tm]) so that every array base is the same for
// the whole wavefront and only the team index varies per lane.  Int arrays are packed (two per FP64 word).
extern __shared__ __align__(16) unsigned char g_lds[];

template <typename T, int EPW>
struct SP {
  int off;  // element offset of the array base (uniform)
  int tm;   // team of this lane
  __device__ __forceinline__ T& operator[](int k) const { return reinterpret_cast<T*>(g_lds)[off + k * EPW + tm]; }
  __device__ __forceinline__ SP operator+(int k) const { return {off + k * EPW, tm}; }
};

template <typename R, int EPW>
struct Ctx {
  using F = SP<R, EPW>;
  using I = SP<int, EPW>;
  F qj, qd, root, F_, L0, vs, o, ax, U, Dinv, Ubar, G, phi, n, x, rbias, rinvA, rlam;
  F q, v, IA, pA, u, tau, arm, W;
  I sact, rkr, misc;
  __device__ __forceinline__ void init(int base, const Lds& L, int tm) {
    // base: offset of the per-environment region in units of R
    constexpr int ratio = (int)(sizeof(R) / sizeof(int));
    auto f = [&](int off) { return F{base + off * EPW, tm}; };
    auto i = [&](int off) { return I{(base + off * EPW) * ratio, tm}; };
    qj = f(L.qj); qd = f(L.qd); root = f(L.root); F_ = f(L.F); L0 = f(L.L0); vs = f(L.vs);
    o = f(L.o); ax = f(L.ax); U = f(L.U); Dinv = f(L.Dinv); Ubar = f(L.Ubar); G = f(L.G);
    phi = f(L.phi); n = f(L.n); x = f(L.x); sact = i(L.sact);
    rkr = i(L.rkr); rbias = f(L.rbias); rinvA = f(L.rinvA); rlam = f(L.rlam); misc = i(L.misc);
    q = f(L.q); v = f(L.v); IA = f(L.IA); pA = f(L.pA); u = f(L.u); tau = f(L.tau); arm = f(L.arm);
    W = f(L.W);
  }
};

// Model tables of one environment template as seen by the kernel: the integer tables of the sweeps
// are LDS copies; slot tables and the float tables are read from global memory (cached).
template <typename R>
struct Tab {
  int n_links, n_actors, n_dof, n_v, n_slots, n_levels, n_anc, r_cap, jfast;
  const int *li, *level_begin, *level_links, *children, *dof_link, *ai;
  const int* anc_link;  // per ancestor entry: link | (column << 16)
  const int *si, *body_slot_begin, *body_slot;
  const double *lf, *sf;
  int n_tj;  // fixed tendons (global memory)
  const int* tj_i;
  const double *tj_f, *tp;
};

// Copies the integer model tables into this workgroup's LDS (all lanes cooperate) and returns the view.
template <typename R>
__device__ __forceinline__ Tab<R> stage_tables(const DevModel& G, R* smem, const Lds& L, int t, int nthreads,
                                              bool copy) {
  // copy = false: the tables of this type are already in LDS (pointers only)
  auto copy_i = [&](int off, const int* src, int n) {
    int* dst = reinterpret_cast<int*>(smem + off);
    if (copy)
      for (int k = t; k < n; k += nthreads) dst[k] = src[k];
    return (const int*)dst;
  };
  Tab<R> T;
  T.n_links = G.n_links; T.n_actors = G.n_actors; T.n_dof = G.n_dof; T.n_v = G.n_v; T.n_slots = G.n_slots;
  T.n_levels = G.n_levels; T.n_anc = G.n_anc; T.r_cap = G.r_cap; T.jfast = G.jfast;
  T.li = copy_i(L.t_li, G.li, G.n_links * LI_COLS);
  T.level_begin = copy_i(L.t_lev, G.level_begin, G.n_levels + 1);
  T.level_links = copy_i(L.t_links, G.level_links, G.n_links);
  T.children = copy_i(L.t_child, G.children, G.n_links - G.n_actors);
  {  // ancestor entries packed as link | (its generalized column << 16): the row responses then index their
     // rows with one LDS read per ancestor instead of two dependent ones
    int* dst = reinterpret_cast<int*>(smem + L.t_anc);
    if (copy)
      for (int k = t; k < G.n_anc; k += nthreads) {
        const int a = G.anc_link[k];
        dst[k] = a | (G.li[a * LI_COLS + LI_COL] << 16);
      }
    T.anc_link = dst;
  }
  T.dof_link = copy_i(L.t_dof, G.dof_link, G.n_dof);
  T.ai = copy_i(L.t_ai, G.ai, G.n_actors * AI_COLS);
  T.si = G.si;
  T.body_slot_begin = G.body_slot_begin;
  T.body_slot = G.body_slot;
  T.lf = G.lf;
  T.sf = G.sf;
  T.n_tj = G.n_tj;
  T.tj_i = G.tj_i;
  T.tj_f = G.tj_f;
  T.tp = G.tp;
  return T;
}

template <typename R>
__device__ __forceinline__ int actor_of_root(const Tab<R>& M, int link) {
  int a = 0;
  for (int k = 0; k < M.n_actors; ++k)
    if (M.ai[k * AI_COLS + AI_ROOT] == link) a = k;
  return a;
}

// clamp to [lo, hi] (lo <= hi): one median-of-three in FP32
__device__ __forceinline__ float clamp_(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
// in FP64 a max then a min, written out: fmin/fmax of loop-carried bounds compile to two more instructions per
// call that quiet signalling NaNs, which no operand here can be
__device__ __forceinline__ double clamp_(double x, double lo, double hi) {
  double r;
  asm("v_max_f64 %0, %1, %2\n\tv_min_f64 %0, %0, %3" : "=&v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}

// upper impulse bound of rows without one (contact normals, limits): far above any impulse, finite so that
// the friction-bound arithmetic of the register Gauss-Seidel stays free of infinities
constexpr double kOpenBound = 1e30;

// bias of a limit or contact-normal row from its position error C: speculative C / h when separated, the
// Baumgarte fraction beta C / h when penetrating
template <typename R>
__device__ __forceinline__ R row_bias(R C, R h, R beta) {
  return C >= R(0) ? C / h : beta * C / h;
}

// rotation matrix (row-major) of a unit quaternion xyzw
template <typename R>
__device__ __forceinline__ void quat_R(R qx, R qy, R qz, R qw, R* M) {
  const R one = R(1), two = R(2);
  M[0] = one - two * (qy * qy + qz * qz); M[1] = two * (qx * qy - qz * qw); M[2] = two * (qx * qz + qy * qw);
  M[3] = two * (qx * qy + qz * qw); M[4] = one - two * (qx * qx + qz * qz); M[5] = two * (qy * qz - qx * qw);
  M[6] = two * (qx * qz - qy * qw); M[7] = two * (qy * qz + qx * qw); M[8] = one - two * (qx * qx + qy * qy);
}
template <typename R, typename P>
__device__ __forceinline__ void quat_R(const P& q, R* M) {
  quat_R(R(q[0]), R(q[1]), R(q[2]), R(q[3]), M);
}

// Pose and velocity of link i (world axes; origin relative to `origin`) from its parent's stored
// orientation (quaternion), origin and velocity and the joint's own position and rate: rotation Rw and
// quaternion qq (xyzw), joint origin o, world joint axis ax (zero at a root), angular velocity w and
// velocity vl of the point o.
// Joint-local parts of every link's pose, which need only the link's own joint coordinate: the joint's
// rotation as a quaternion (axis sin(q/2), cos(q/2); identity for a prismatic joint) into q, the joint anchor
// in the parent frame (moved along the axis by a prismatic coordinate) into o, the local axis into ax.  The
// level-by-level sweep then only composes them with the parent's pose, and the sines and cosines of all
// joints are taken at once instead of one tree level after the other.
template <typename R, int EPW, int TEAM>
__device__ __forceinline__ void stage_joint_locals(const Tab<R>& M, const Ctx<R, EPW>& s, int tt) {
  for (int i = tt; i < M.n_links; i += TEAM) {
    const int* li = M.li + i * LI_COLS;
    const int jt = li[LI_JTYPE];
    if (jt != J_REV && jt != J_PRI) continue;
    const double* lf = M.lf + i * LF_COLS;
    const V3<R> axl = ld3<R>(lf + LF_AXIS);
    V3<R> tl = ld3<R>(lf + LF_ANCHOR);
    const R q = s.qj[li[LI_DOF]];
    R lq[4] = {R(0), R(0), R(0), R(1)};
    if (jt == J_REV) {
      R sh, ch;
      sincos_(R(0.5) * q, &sh, &ch);
      lq[0] = axl.x * sh;
      lq[1] = axl.y * sh;
      lq[2] = axl.z * sh;
      lq[3] = ch;
    } else {
      tl = add(tl, mul(axl, q));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s.q[4 * i + k] = lq[k];
    st3(s.o + 3 * i, tl);
    st3(s.ax + 3 * i, axl);
  }
}

template <typename R, int EPW>
__device__ __forceinline__ void link_kinematics(const Tab<R>& M, const Ctx<R, EPW>& s, int i, V3<R> origin, R* Rw,
                                                R* qq, V3<R>& o, V3<R>& w, V3<R>& vl, V3<R>& ax, bool root_level) {
  // root_level: the links of tree level 0, the roots; every deeper link has a one-DOF joint
  const int* li = M.li + i * LI_COLS;
  const int jt = li[LI_JTYPE];
  ax = mk(R(0), R(0), R(0));
  if (root_level) {
    // root pose from the root state (quaternion xyzw, normalised on read)
    const auto rs = s.root + 13 * actor_of_root(M, i);
    const R qx = rs[3], qy = rs[4], qz = rs[5], qw = rs[6];
    const R inv = rsqrt_(qx * qx + qy * qy + qz * qz + qw * qw);
    qq[0] = qx * inv; qq[1] = qy * inv; qq[2] = qz * inv; qq[3] = qw * inv;
    quat_R(qq[0], qq[1], qq[2], qq[3], Rw);
    o = sub(ld3<R>(rs), origin);
    if (jt == J_FREE) {
      const int c = li[LI_ROOTCOL];
      vl = ld3<R>(s.qd + c);
      w = ld3<R>(s.qd + c + 3);
    } else {
      vl = mk(R(0), R(0), R(0));
      w = vl;
    }
    return;
  }
  // the joint's local rotation, anchor and axis, staged by stage_joint_locals
  const int p = li[LI_PARENT];
  const auto qp = s.q + 4 * p;
  const R px = qp[0], py = qp[1], pz = qp[2], pw = qp[3];
  R Rp[9];
  quat_R(px, py, pz, pw, Rp);
  const V3<R> axl = ld3<R>(s.ax + 3 * i);
  const V3<R> tl = ld3<R>(s.o + 3 * i);
  const R rx = s.q[4 * i], ry = s.q[4 * i + 1], rz = s.q[4 * i + 2], ch = s.q[4 * i + 3];
  const R qd = s.qd[li[LI_COL]];
  if (jt == J_REV) {
    // parent orientation composed with the joint rotation (angle q about the local axis)
    qq[0] = pw * rx + ch * px + (py * rz - pz * ry);
    qq[1] = pw * ry + ch * py + (pz * rx - px * rz);
    qq[2] = pw * rz + ch * pz + (px * ry - py * rx);
    qq[3] = pw * ch - (px * rx + py * ry + pz * rz);
    quat_R(qq[0], qq[1], qq[2], qq[3], Rw);
  } else {
    qq[0] = px; qq[1] = py; qq[2] = pz; qq[3] = pw;
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = Rp[k];
  }
  ax = mv(Rp, axl);
  const V3<R> op = ld3<R>(s.o + 3 * p);
  o = add(op, mv(Rp, tl));
  w = ld3<R>(s.v + 6 * p);
  vl = add(ld3<R>(s.v + 6 * p + 3), cross(w, sub(o, op)));
  if (jt == J_REV) w = add(w, mul(ax, qd));
  else vl = add(vl, mul(ax, qd));
}

// velocity-product acceleration of a joint (world axes about the joint origin), from the link's velocity
// (w, v at o) after the joint's own motion: revolute ((w x s) qd, (v x s) qd), prismatic (0, (w x s) qd)
template <typename R, int EPW>
__device__ __forceinline__ void vel_product(const Ctx<R, EPW>& s, int i, int jt, V3<R> ax, R qd, V3<R>& ca, V3<R>& cl) {
  const V3<R> w = ld3<R>(s.v + 6 * i), vl = ld3<R>(s.v + 6 * i + 3);
  if (jt == J_REV) {
    ca = mul(cross(w, ax), qd);
    cl = mul(cross(vl, ax), qd);
  } else {
    ca = mk(R(0), R(0), R(0));
    cl = mul(cross(w, ax), qd);
  }
}

// Adds the joint loads of one unit test load to Wrow (u_k at each joint column on the path of link k)
// and the resulting bias force at a free root ([n; f] in the root's 6 columns).  The load is a spatial
// force given by its bias contribution (pn, pf) = -f about o_k, or a joint force tau0 at link k.
template <typename R, int EPW, typename WP>
__device__ __forceinline__ void unit_load_inward(const Tab<R>& M, const Ctx<R, EPW>& s, int k, V3<R> pn, V3<R> pf, R tau0,
                                 const WP& Wrow) {
  while (true) {
    const int* li = M.li + k * LI_COLS;
    const int jt = li[LI_JTYPE];
    if (jt == J_FIXED) return;
    if (jt == J_FREE) {
      const int c = li[LI_ROOTCOL];
      Wrow[c + 0] += pn.x; Wrow[c + 1] += pn.y; Wrow[c + 2] += pn.z;
      Wrow[c + 3] += pf.x; Wrow[c + 4] += pf.y; Wrow[c + 5] += pf.z;
      return;
    }
    const V3<R> ax = ld3<R>(s.ax + 3 * k);
    const V3<R> Ua = ld3<R>(s.U + 6 * k), Ul = ld3<R>(s.U + 6 * k + 3);
    const R u = tau0 - (jt == J_REV ? dot(ax, pn) : dot(ax, pf));
    tau0 = R(0);
    Wrow[li[LI_COL]] += u;
    const R ud = u * s.Dinv[k];
    pn = add(pn, mul(Ua, ud));
    pf = add(pf, mul(Ul, ud));
    const int p = li[LI_PARENT];
    pn = add(pn, cross(sub(ld3<R>(s.o + 3 * k), ld3<R>(s.o + 3 * p)), pf));
    k = p;
  }
}

// Row of a point load along d at point x on link k (sign +-1): adds J entries to Jrow when non-null and
// returns sum_j J_j Wrow_j when Wrow is non-null.
template <typename R, int EPW, typename JP, typename WP>
__device__ __forceinline__ R point_row(const Tab<R>& M, const Ctx<R, EPW>& s, int k, V3<R> x, V3<R> d, R sign, const JP& Jrow,
                       const WP& Wrow, bool want_j, bool want_w) {
  R acc = R(0);
  while (true) {
    const int* li = M.li + k * LI_COLS;
    const int jt = li[LI_JTYPE];
    if (jt == J_FIXED) break;
    if (jt == J_FREE) {
      const int c = li[LI_ROOTCOL];
      const V3<R> mo = cross(sub(x, ld3<R>(s.o + 3 * k)), d);
      const R j6[6] = {d.x, d.y, d.z, mo.x, mo.y, mo.z};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        if (want_j) Jrow[c + q] += sign * j6[q];
        if (want_w) acc += sign * j6[q] * Wrow[c + q];
      }
      break;
    }
    const V3<R> ax = ld3<R>(s.ax + 3 * k);
    const R jv = jt == J_REV ? dot(ax, cross(sub(x, ld3<R>(s.o + 3 * k)), d)) : dot(ax, d);
    const int c = li[LI_COL];
    if (want_j) Jrow[c] += sign * jv;
    if (want_w) acc += sign * jv * Wrow[c];
    k = li[LI_PARENT];
  }
  return acc;
}


// Compact Jacobian row of a constraint: its entries on the free-root columns of the two bodies' articulations
// (6 each, about the root's point) and on up to kJointEntries joint columns; unused entries are zero.
template <typename R>
struct JRow {
  int ra, rb;  // first root column of body a / body b, -1 if none
  R ja[6], jb[6];
  int c[kJointEntries];
  R val[kJointEntries];
};

template <typename R>
__device__ __forceinline__ void jrow_clear(JRow<R>& J) {
  J.ra = -1;
  J.rb = -1;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    J.ja[q] = R(0);
    J.jb[q] = R(0);
  }
#pragma unroll
  for (int e = 0; e < kJointEntries; ++e) {
    J.c[e] = 0;
    J.val[e] = R(0);
  }
}

// sum_j J_j w_j
template <typename R, typename WP>
__device__ __forceinline__ R jrow_dot(const JRow<R>& J, const WP& w) {
  // two partial sums: a chain of 11 fused multiply-adds instead of 22
  R a[2] = {R(0), R(0)};
#pragma unroll
  for (int e = 0; e < kJointEntries; ++e) a[e & 1] += J.val[e] * w[J.c[e]];
  if (J.ra >= 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) a[q & 1] += J.ja[q] * w[J.ra + q];
  }
  if (J.rb >= 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) a[(q + 1) & 1] += J.jb[q] * w[J.rb + q];
  }
  return a[0] + a[1];
}

// root part of a point load along d at x on the articulation of link k: sign (d, (x - o_root) x d)
template <typename R, int EPW>
__device__ __forceinline__ int jrow_root(const Tab<R>& M, const Ctx<R, EPW>& s, int k, V3<R> x, V3<R> d, R sign, R* j6) {
  const int* li = M.li + k * LI_COLS;
  const int rc = li[LI_ROOTCOL];
  const V3<R> mo = cross(sub(x, ld3<R>(s.o + 3 * li[LI_ROOT])), d);
  const bool on = rc >= 0;
  j6[0] = on ? sign * d.x : R(0); j6[1] = on ? sign * d.y : R(0); j6[2] = on ? sign * d.z : R(0);
  j6[3] = on ? sign * mo.x : R(0); j6[4] = on ? sign * mo.y : R(0); j6[5] = on ? sign * mo.z : R(0);
  return rc;
}

// Row of a point load along d at x between link ka (+) and link kb (-, or none when kb < 0).  The joint
// entries of ka's path to its root come first, then kb's; the walk is unrolled so the row stays in registers.
template <typename R, int EPW>
__device__ __forceinline__ void jrow_point(const Tab<R>& M, const Ctx<R, EPW>& s, int ka, int kb, V3<R> x, V3<R> d,
                                           JRow<R>& J) {
  J.ra = jrow_root(M, s, ka, x, d, R(1), J.ja);
  if (kb >= 0) {
    J.rb = jrow_root(M, s, kb, x, d, R(-1), J.jb);
  } else {
    J.rb = -1;
#pragma unroll
    for (int q = 0; q < 6; ++q) J.jb[q] = R(0);
  }
  int k = ka;
  R sg = R(1);
  bool onb = false;
#pragma unroll
  for (int e = 0; e < kJointEntries; ++e) {
    int jt = k >= 0 ? M.li[k * LI_COLS + LI_JTYPE] : J_FIXED;
    if (jt != J_REV && jt != J_PRI && !onb) {  // body a's path ended: continue on body b's
      onb = true;
      k = kb;
      sg = R(-1);
      jt = k >= 0 ? M.li[k * LI_COLS + LI_JTYPE] : J_FIXED;
    }
    J.c[e] = 0;
    J.val[e] = R(0);
    if (jt == J_REV || jt == J_PRI) {
      const int* li = M.li + k * LI_COLS;
      const V3<R> ax = ld3<R>(s.ax + 3 * k);
      const R jv = jt == J_REV ? dot(ax, cross(sub(x, ld3<R>(s.o + 3 * k)), d)) : dot(ax, d);
      J.c[e] = li[LI_COL];
      J.val[e] = sg * jv;
      k = li[LI_PARENT];
    }
  }
}

}  // namespace

// One env-step of the environments of group `group` of type T (EPW environments per wavefront).
// stage: copy T's model tables into LDS (false when the previous group of this workgroup had the same type).
// TGS: the temporal Gauss-Seidel variant (a separate instantiation, so that the default solver's registers
// are not shared with the variant's extra per-row state).
template <typename R, int TEAM, bool TGS, bool CYC>
__device__ __forceinline__ void step_group(const StepArgs& P, const TypeArgs& T, int group, bool stage) {
  R* smem = reinterpret_cast<R*>(g_lds);
  const Lds& L = T.lds;
  const int n_envs = T.n_envs;
  constexpr int EPW = kTeam / TEAM;  // environments per wavefront
  constexpr int FR = kFastRows;      // rows of the register Gauss-Seidel path and of one response chunk
  constexpr int kWideAhead = 8;      // wide path: rows of A columns in flight ahead of the Gauss-Seidel updates
  static_assert(FR <= TEAM, "fast rows exceed the lanes of an environment");
  const int t = threadIdx.x;         // lane in the wavefront
  const int tm = EPW == 1 ? 0 : t / TEAM;  // team (environment slot) of this lane
  const int tt = EPW == 1 ? t : t % TEAM;  // lane within the team
  const int gidx = group * EPW + tm;
  const bool valid = gidx < n_envs;  // the last wavefront's spare teams recompute an env but write nothing
  const int env = T.env_list[valid ? gidx : n_envs - 1];
  const Tab<R> M = stage_tables<R>(T.m, smem, L, t, kTeam, stage);
  Ctx<R, EPW> s;
  s.init(L.team_base, L, tm);
  __syncthreads();

  const int nl = M.n_links, nd = M.n_dof, nv = M.n_v, ns = M.n_slots, na = M.n_actors;
  const int abase = P.env_actor_base[env], dbase = P.env_dof_base[env], bbase = P.env_body_base[env];
  const R h = R(P.h);
  constexpr bool tgs = TGS;
  R* Jg = reinterpret_cast<R*>(T.scratch) + (long long)gidx * T.scratch_stride;
  R* Wg = Jg + (long long)M.r_cap * nv;
  R* Ag = Wg + (long long)M.r_cap * nv;  // wide path: columns of A, TEAM entries per row

  // ---------------------------------------------------------------- load state
  for (int k = tt; k < 13 * na; k += TEAM) s.root[k] = R(P.root_state[(long long)abase * 13 + k]);
  for (int j = tt; j < nd; j += TEAM) {
    const int lk = M.dof_link[j];
    s.qj[j] = R(P.dof_state[2ll * (dbase + j)]);
    s.qd[M.li[lk * LI_COLS + LI_COL]] = R(P.dof_state[2ll * (dbase + j) + 1]);
  }
  for (int k = tt; k < 3 * nl; k += TEAM) s.F_[k] = R(0);
  __syncthreads();
  for (int k = tt; k < na; k += TEAM) {
    const int* ai = M.ai + k * AI_COLS;
    if (!ai[AI_FIXED])
      for (int q = 0; q < 6; ++q) s.qd[ai[AI_COL] + q] = s.root[13 * k + 7 + q];
  }
  R dof_force_acc = R(0);
  bool slow_any = false;  // some substep took the row-response slow path
  int rows_max = 0;       // most rows of a substep
  __syncthreads();
  const V3<R> origin = ld3<R>(s.root);
  // optional per-phase clock accounting (lane 0), compiled only into the instantiation launched when the
  // debug tensor is bound: the counters would otherwise hold registers through the whole kernel
  long long cyc[kPhases] = {0};
  int cur_phase = -1;
  long long t_mark = 0;
#define PHASE_MARK(ph)                                              \
  if (CYC) {                                                        \
    const long long now = (long long)clock64();                     \
    if (cur_phase >= 0) cyc[cur_phase] += now - t_mark;             \
    cur_phase = (ph);                                               \
    t_mark = now;                                                   \
  }

  for (int sub_i = 0; sub_i < P.substeps; ++sub_i) {
    PHASE_MARK(0);
    // ---------------------------------------------------- controls: actuation + implicit PD drive
    // the drive kp (q* - q+) + kd (qd* - qd+) at the end of the substep splits into an explicit part
    // and the armature h kd + h^2 kp added to the joint's diagonal of M~
    for (int j = tt; j < nd; j += TEAM) {
      const int lk = M.dof_link[j];
      const double* lf = M.lf + lk * LF_COLS;
      const int c = M.li[lk * LI_COLS + LI_COL];
      const R pt = P.pos_tgt ? R(P.pos_tgt[dbase + j]) : R(0);
      const R vt = P.vel_tgt ? R(P.vel_tgt[dbase + j]) : R(0);
      const R kp = R(P.dof_kp ? double(P.dof_kp[dbase + j]) : lf[LF_KP]);
      const R kd = R(P.dof_kd ? double(P.dof_kd[dbase + j]) : lf[LF_KD]);
      s.tau[c] = R(P.act[dbase + j]) + kp * (pt - s.qj[j] - h * s.qd[c]) + kd * (vt - s.qd[c]);
      s.arm[c] = R(lf[LF_ARM]) + h * kd + h * h * kp;
    }
    __syncthreads();
    if (M.n_tj > 0) {
      // fixed tendons, explicit: lengths and rates down each tendon tree (one lane per env; the articulated
      // inertia region is free until the forward sweep), then every tendon joint's spring, damper and limit
      // force on the DOFs of its path as -f coef
      if (tt == 0) {
        const auto len = s.IA;
        const auto rate = s.IA + M.n_tj;
        for (int j = 0; j < M.n_tj; ++j) {
          const int* ti = M.tj_i + 4 * j;
          const R cf = R(M.tj_f[j]);
          len[j] = (ti[3] >= 0 ? len[ti[3]] : R(0)) + cf * s.qj[ti[1]];
          rate[j] = (ti[3] >= 0 ? rate[ti[3]] : R(0)) + cf * s.qd[ti[2]];
        }
        for (int j = 0; j < M.n_tj; ++j) {
          const double* tp = M.tp + 6 * M.tj_i[4 * j];
          const R l = len[j];
          R f = R(tp[0]) * (l - R(tp[2])) + R(tp[1]) * rate[j];
          if (l > R(tp[4])) f += R(tp[5]) * (l - R(tp[4]));
          if (l < R(tp[3])) f += R(tp[5]) * (l - R(tp[3]));
          for (int p = j; p >= 0; p = M.tj_i[4 * p + 3]) s.tau[M.tj_i[4 * p + 2]] -= f * R(M.tj_f[p]);
        }
      }
      __syncthreads();
    }

    PHASE_MARK(1);
    // ---------------------------------------------------- forward sweep by depth
    // Poses and velocities chain from parent to child, level by level; the spatial inertia and bias force
    // of each link need only its own pose and velocity, so they are formed afterwards for all links at
    // once (lanes over links) instead of by the one or two lanes a level occupies.
    stage_joint_locals<R, EPW, TEAM>(M, s, tt);
    __syncthreads();
    for (int d = 0; d < M.n_levels; ++d) {
      for (int idx = M.level_begin[d] + tt; idx < M.level_begin[d + 1]; idx += TEAM) {
        const int i = M.level_links[idx];
        R Rw[9], qq[4];
        V3<R> o, w, vl, ax;
        link_kinematics(M, s, i, origin, Rw, qq, o, w, vl, ax, d == 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) s.q[4 * i + k] = qq[k];
        st3(s.o + 3 * i, o);
        st3(s.ax + 3 * i, ax);
        st3(s.v + 6 * i, w);
        st3(s.v + 6 * i + 3, vl);
      }
      __syncthreads();
    }
    for (int i = tt; i < nl; i += TEAM) {
      const double* lf = M.lf + i * LF_COLS;
      R Rw[9];
      quat_R(s.q + 4 * i, Rw);
      const V3<R> w = ld3<R>(s.v + 6 * i), vl = ld3<R>(s.v + 6 * i + 3);
      // spatial inertia about o (world axes): A = Ic_w + m (|d|^2 1 - d d^T), B = m d^, M = m 1
      const double msc = P.mass_scale ? double(P.mass_scale[bbase + i]) : 1.0;  // per-env mass factor
      const R m = R(lf[LF_MASS] * msc);
      const V3<R> d = mv(Rw, ld3<R>(lf + LF_COM));
      const double* Icl = lf + LF_IC;
      const R Ic[9] = {R(Icl[0] * msc), R(Icl[3] * msc), R(Icl[4] * msc), R(Icl[3] * msc), R(Icl[1] * msc),
                       R(Icl[5] * msc), R(Icl[4] * msc), R(Icl[5] * msc), R(Icl[2] * msc)};
      R Tm[9], Iw[9];
      mm3(Rw, Ic, Tm);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          Iw[3 * a + b] = Tm[3 * a] * Rw[3 * b] + Tm[3 * a + 1] * Rw[3 * b + 1] + Tm[3 * a + 2] * Rw[3 * b + 2];
      SI<R> I;
      const R dd = dot(d, d), half = R(0.5);
      I.A[0] = Iw[0] + m * (dd - d.x * d.x);
      I.A[1] = Iw[4] + m * (dd - d.y * d.y);
      I.A[2] = Iw[8] + m * (dd - d.z * d.z);
      I.A[3] = half * (Iw[1] + Iw[3]) - m * d.x * d.y;
      I.A[4] = half * (Iw[2] + Iw[6]) - m * d.x * d.z;
      I.A[5] = half * (Iw[5] + Iw[7]) - m * d.y * d.z;
      I.B[0] = R(0); I.B[1] = -m * d.z; I.B[2] = m * d.y;
      I.B[3] = m * d.z; I.B[4] = R(0); I.B[5] = -m * d.x;
      I.B[6] = -m * d.y; I.B[7] = m * d.x; I.B[8] = R(0);
      I.M[0] = m; I.M[1] = m; I.M[2] = m; I.M[3] = R(0); I.M[4] = R(0); I.M[5] = R(0);
      // bias force p = v x* (I v) - f_gravity (gravity m g at the COM)
      V3<R> ha, hl;
      si_mul(I, w, vl, ha, hl);
      // gravity of this env, read where it is used (a per-env value held across the substep loop would cost
      // registers the kernel does not have)
      const V3<R> grav = P.env_gravity ? mk(R(P.env_gravity[3 * env]), R(P.env_gravity[3 * env + 1]), R(P.env_gravity[3 * env + 2]))
                                       : mk(R(P.gx), R(P.gy), R(P.gz));
      const V3<R> fg = mul(grav, m);
      const V3<R> pn = sub(add(cross(w, ha), cross(vl, hl)), cross(d, fg));
      const V3<R> pf = sub(cross(w, hl), fg);
      si_store(I, s.IA + 21 * i);
      st3(s.pA + 6 * i, pn);
      st3(s.pA + 6 * i + 3, pf);
    }
    __syncthreads();

    PHASE_MARK(2);
    // ---------------------------------------------------- ABA inward sweep (deepest level first)
    if constexpr (TEAM == 64) {
      // Up to three links of a level at a time, 21 lanes each, one per stored entry of the 6x6 articulated
      // inertia (A: xx yy zz xy xz yz, B row-major, M: xx yy zz xy xz yz).  Per link: (1) every entry lane adds
      // the children's entry (lanes 0-5 also the bias force), (2) every lane of the link forms U = I^A S, D,
      // 1/D, u and the articulated bias force moved to the parent's origin (its lane 0 stores them), (3) every
      // entry lane forms its entry of X^T (I^A - U U^T / D) X, X moving the inertia from o_i to o_parent, from
      // the nine entries of I^A it combines.  The per-link work of one lane shrinks from the whole 6x6 update
      // and move to its own entry.
      const int slot = tt / 21, el = tt - 21 * slot;
      int ep, eq;  // the lane's entry (ep, eq)
      if (el < 6) {
        ep = el < 3 ? el : (el == 5 ? 1 : 0);
        eq = el < 3 ? el : (el == 3 ? 1 : 2);
      } else if (el < 15) {
        ep = (el - 6) / 3;
        eq = 3 + (el - 6) % 3;
      } else {
        const int k = el - 15;
        ep = 3 + (k < 3 ? k : (k == 5 ? 1 : 0));
        eq = 3 + (k < 3 ? k : (k == 3 ? 1 : 2));
      }
      // rows of X in column p: p itself and, for an angular p, the linear rows 3 + (p+1)%3 (coefficient
      // -r[(p+2)%3]) and 3 + (p+2)%3 (coefficient r[(p+1)%3])
      const int mr[3] = {ep, ep < 3 ? 3 + (ep + 1) % 3 : ep, ep < 3 ? 3 + (ep + 2) % 3 : ep};
      const int nc[3] = {eq, eq < 3 ? 3 + (eq + 1) % 3 : eq, eq < 3 ? 3 + (eq + 2) % 3 : eq};
      for (int d = M.n_levels - 1; d >= 0; --d) {
        const int lb = M.level_begin[d], le = M.level_begin[d + 1];
        for (int b0 = lb; b0 < le; b0 += 3) {
          const int idx = b0 + slot;
          const bool act = slot < 3 && idx < le;
          const int i = act ? M.level_links[idx] : 0;
          const int* li = M.li + i * LI_COLS;
          const int jt = act ? li[LI_JTYPE] : J_FIXED;
          if (jt != J_FIXED) {  // (1) children hold I^a, p^a moved to o_i
            R a = s.IA[21 * i + el];
            R pa = el < 6 ? s.pA[6 * i + el] : R(0);
            for (int q = li[LI_CHILD_BEGIN]; q < li[LI_CHILD_END]; ++q) {
              const int ch = M.children[q];
              a += s.IA[21 * ch + el];
              if (el < 6) pa += s.pA[6 * ch + el];
            }
            s.IA[21 * i + el] = a;
            if (el < 6) s.pA[6 * i + el] = pa;
          }
          __syncthreads();
          if (jt == J_FREE && el == 0) {
            SI<R> I;
            si_load(I, s.IA + 21 * i);
            const int a = actor_of_root(M, i);
            chol6(I, s.L0 + 27 * a, s.L0 + 27 * a + 21);
          }
          const bool one = jt == J_REV || jt == J_PRI;  // a one-DOF joint
          R Dinv = R(0);
          V3<R> r = mk(R(0), R(0), R(0));
          if (one) {  // (2)
            SI<R> I;
            si_load(I, s.IA + 21 * i);
            const V3<R> pn = ld3<R>(s.pA + 6 * i), pf = ld3<R>(s.pA + 6 * i + 3);
            const int c = li[LI_COL];
            const V3<R> ax = ld3<R>(s.ax + 3 * i);
            V3<R> Ua, Ul;
            R D, u;
            if (jt == J_REV) {
              Ua = symv(I.A, ax);
              Ul = mtv(I.B, ax);
              D = dot(ax, Ua);
              u = s.tau[c] - dot(ax, pn);
            } else {
              Ua = mv(I.B, ax);
              Ul = symv(I.M, ax);
              D = dot(ax, Ul);
              u = s.tau[c] - dot(ax, pf);
            }
            D += s.arm[c];
            Dinv = R(1) / D;
            // p^a = p^A + I^a c + U u / D = p^A + I^A c + U (u - U . c) / D, then moved to the parent's origin
            V3<R> ca, cl, ia, il;
            vel_product(s, i, jt, ax, s.qd[c], ca, cl);
            si_mul(I, ca, cl, ia, il);
            const R g = (u - dot(Ua, ca) - dot(Ul, cl)) * Dinv;
            const V3<R> pfa = add(add(pf, il), mul(Ul, g));
            r = sub(ld3<R>(s.o + 3 * i), ld3<R>(s.o + 3 * li[LI_PARENT]));
            const V3<R> pna = add(add(add(pn, ia), mul(Ua, g)), cross(r, pfa));
            if (el == 0) {
              st3(s.pA + 6 * i, pna);
              st3(s.pA + 6 * i + 3, pfa);
              st3(s.U + 6 * i, Ua);
              st3(s.U + 6 * i + 3, Ul);
              s.Dinv[i] = Dinv;
              s.u[i] = u;
            }
          }
          __syncthreads();
          R val = R(0);
          if (one) {  // (3)
            // all fifteen reads first, then the arithmetic
            R um[3], un[3], ia[9];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              um[a] = s.U[6 * i + mr[a]];
              un[a] = s.U[6 * i + nc[a]];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b = 0; b < 3; ++b) ia[3 * a + b] = s.IA[21 * i + si_index(mr[a], nc[b])];
            // coefficients: -r[(p+2)%3] and r[(p+1)%3] for an angular p, by selects on p
            const R rp1 = ep == 0 ? r.z : (ep == 1 ? r.x : r.y), rp2 = ep == 0 ? r.y : (ep == 1 ? r.z : r.x);
            const R rq1 = eq == 0 ? r.z : (eq == 1 ? r.x : r.y), rq2 = eq == 0 ? r.y : (eq == 1 ? r.z : r.x);
            const R xp[3] = {R(1), ep < 3 ? -rp1 : R(0), ep < 3 ? rp2 : R(0)};
            const R xq[3] = {R(1), eq < 3 ? -rq1 : R(0), eq < 3 ? rq2 : R(0)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              R acc = R(0);
#pragma unroll
              for (int b = 0; b < 3; ++b) acc += xq[b] * (ia[3 * a + b] - um[a] * un[b] * Dinv);
              val += xp[a] * acc;
            }
          }
          __syncthreads();
          if (one) s.IA[21 * i + el] = val;
          __syncthreads();
        }
      }
    } else {
      for (int d = M.n_levels - 1; d >= 0; --d) {
        for (int idx = M.level_begin[d] + tt; idx < M.level_begin[d + 1]; idx += TEAM) {
          const int i = M.level_links[idx];
          const int* li = M.li + i * LI_COLS;
          const int jt = li[LI_JTYPE];
          if (jt == J_FIXED) continue;
          SI<R> I;
          si_load(I, s.IA + 21 * i);
          V3<R> pn = ld3<R>(s.pA + 6 * i), pf = ld3<R>(s.pA + 6 * i + 3);
          for (int q = li[LI_CHILD_BEGIN]; q < li[LI_CHILD_END]; ++q) {  // children hold I^a, p^a moved to o_i
            const int ch = M.children[q];
            si_addload(I, s.IA + 21 * ch);
            pn = add(pn, ld3<R>(s.pA + 6 * ch));
            pf = add(pf, ld3<R>(s.pA + 6 * ch + 3));
          }
          if (jt == J_FREE) {
            st3(s.pA + 6 * i, pn);
            st3(s.pA + 6 * i + 3, pf);
            const int a = actor_of_root(M, i);
            chol6(I, s.L0 + 27 * a, s.L0 + 27 * a + 21);
            continue;
          }
          const int c = li[LI_COL];
          const V3<R> ax = ld3<R>(s.ax + 3 * i);
          V3<R> Ua, Ul;
          R D, u;
          if (jt == J_REV) {
            Ua = symv(I.A, ax);
            Ul = mtv(I.B, ax);
            D = dot(ax, Ua);
            u = s.tau[c] - dot(ax, pn);
          } else {
            Ua = mv(I.B, ax);
            Ul = symv(I.M, ax);
            D = dot(ax, Ul);
            u = s.tau[c] - dot(ax, pf);
          }
          D += s.arm[c];
          const R Dinv = R(1) / D;
          // I^a = I^A - U U^T / D
          I.A[0] -= Ua.x * Ua.x * Dinv; I.A[1] -= Ua.y * Ua.y * Dinv; I.A[2] -= Ua.z * Ua.z * Dinv;
          I.A[3] -= Ua.x * Ua.y * Dinv; I.A[4] -= Ua.x * Ua.z * Dinv; I.A[5] -= Ua.y * Ua.z * Dinv;
          I.M[0] -= Ul.x * Ul.x * Dinv; I.M[1] -= Ul.y * Ul.y * Dinv; I.M[2] -= Ul.z * Ul.z * Dinv;
          I.M[3] -= Ul.x * Ul.y * Dinv; I.M[4] -= Ul.x * Ul.z * Dinv; I.M[5] -= Ul.y * Ul.z * Dinv;
          const R ua[3] = {Ua.x, Ua.y, Ua.z}, ul[3] = {Ul.x, Ul.y, Ul.z};
  #pragma unroll
          for (int a = 0; a < 3; ++a)
  #pragma unroll
            for (int b = 0; b < 3; ++b) I.B[3 * a + b] -= ua[a] * ul[b] * Dinv;
          // p^a = p^A + I^a c + U u / D
          V3<R> ca, cl, ia, il;
          vel_product(s, i, jt, ax, s.qd[c], ca, cl);
          si_mul(I, ca, cl, ia, il);
          const R ud = u * Dinv;
          pn = add(add(pn, ia), mul(Ua, ud));
          pf = add(add(pf, il), mul(Ul, ud));
          // move to the parent's point (nothing to move for a joint anchored at its parent's origin, such as the
          // massless links of per-axis joint chains)
          const V3<R> r = sub(ld3<R>(s.o + 3 * i), ld3<R>(s.o + 3 * li[LI_PARENT]));
          if (r.x != R(0) || r.y != R(0) || r.z != R(0)) {
            si_shift(I, r);
            pn = add(pn, cross(r, pf));
          }
          si_store(I, s.IA + 21 * i);
          st3(s.pA + 6 * i, pn);
          st3(s.pA + 6 * i + 3, pf);
          st3(s.U + 6 * i, Ua);
          st3(s.U + 6 * i + 3, Ul);
          s.Dinv[i] = Dinv;
          s.u[i] = u;
        }
        __syncthreads();
      }

    }

    PHASE_MARK(3);
    // ---------------------------------------------------- root solve and ABA outward sweep
    // link accelerations overwrite the (consumed) bias forces: a_i lives in pA_i.  Level 0 holds the roots
    // and every deeper link has a one-DOF joint, so the deeper levels read all their operands at once and
    // do not branch on the joint type.
    for (int d = 0; d < M.n_levels; ++d) {
      for (int idx = M.level_begin[d] + tt; idx < M.level_begin[d + 1]; idx += TEAM) {
        const int i = M.level_links[idx];
        const int* li = M.li + i * LI_COLS;
        V3<R> aa, al;
        if (d == 0) {
          const int jt = li[LI_JTYPE];
          aa = mk(R(0), R(0), R(0));
          al = aa;
          if (jt == J_FREE) {
            const int a = actor_of_root(M, i);
            R x[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) x[q] = -s.pA[6 * i + q];
            chol6_solve(s.L0 + 27 * a, s.L0 + 27 * a + 21, x);
            aa = mk(x[0], x[1], x[2]);
            al = mk(x[3], x[4], x[5]);
            // classical acceleration of the centre of mass: a_lin + w x v_com
            const int c = li[LI_ROOTCOL];
            st3(s.vs + c, add(al, cross(ld3<R>(s.qd + c + 3), ld3<R>(s.qd + c))));
            st3(s.vs + c + 3, aa);
          }
        } else {
          const int jt = li[LI_JTYPE], p = li[LI_PARENT], c = li[LI_COL];
          const bool rev = jt == J_REV;
          const V3<R> r = sub(ld3<R>(s.o + 3 * i), ld3<R>(s.o + 3 * p));
          const V3<R> ax = ld3<R>(s.ax + 3 * i);
          const V3<R> w = ld3<R>(s.v + 6 * i), vl = ld3<R>(s.v + 6 * i + 3);
          const R qd = s.qd[c];
          const V3<R> pa = ld3<R>(s.pA + 6 * p), pl = ld3<R>(s.pA + 6 * p + 3);
          const V3<R> Ua = ld3<R>(s.U + 6 * i), Ul = ld3<R>(s.U + 6 * i + 3);
          const R ui = s.u[i], dinv = s.Dinv[i];
          // velocity product: revolute ((w x s) qd, (v x s) qd), prismatic (0, (w x s) qd)
          const V3<R> wxs = mul(cross(w, ax), qd), vxs = mul(cross(vl, ax), qd);
          const V3<R> ca = rev ? wxs : mk(R(0), R(0), R(0)), cl = rev ? vxs : wxs;
          aa = add(pa, ca);
          al = add(add(pl, cross(pa, r)), cl);
          const R qdd = (ui - dot(Ua, aa) - dot(Ul, al)) * dinv;
          if (rev) aa = add(aa, mul(ax, qdd));
          else al = add(al, mul(ax, qdd));
          s.vs[c] = qdd;
        }
        st3(s.pA + 6 * i, aa);
        st3(s.pA + 6 * i + 3, al);
      }
      __syncthreads();
    }
    // free accelerations (debug) and v* = qd + h qdd_free, in place
    for (int c = tt; c < nv; c += TEAM) {
      const R qdd = s.vs[c];
      if (P.dbg_qdd && valid) P.dbg_qdd[(long long)env * P.dbg_qdd_stride + sub_i * P.dbg_qdd_sub + c] = float(qdd);
      s.vs[c] = s.qd[c] + h * qdd;
    }
    __syncthreads();

    PHASE_MARK(4);
    // ---------------------------------------------------- link velocities under v*, U about roots, G table
    // U about the root point and the G table need only the inward sweep's results, so every link forms its
    // own at once (lanes over links); the velocities chain level by level.
    for (int i = tt; i < nl; i += TEAM) {
      const int* li = M.li + i * LI_COLS;
      if (li[LI_PARENT] < 0) continue;
      // U moved to the root point (its linear half is unchanged), and G_ik = U_i . (s_k moved to o_i)
      // for every ancestor joint k
      const V3<R> oi = ld3<R>(s.o + 3 * i);
      const V3<R> Ua = ld3<R>(s.U + 6 * i), Ul = ld3<R>(s.U + 6 * i + 3);
      st3(s.Ubar + 3 * i, add(Ua, cross(sub(oi, ld3<R>(s.o + 3 * li[LI_ROOT])), Ul)));
      // four ancestors at a time, their reads issued together (entries past the last one recompute the
      // last one's value)
      const int qb = li[LI_ANC_BEGIN], qe = li[LI_ANC_END];
      for (int q0 = qb; q0 < qe; q0 += 4) {
        R gv[4];
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
          const int k = M.anc_link[min(q0 + k4, qe - 1)] & 0xffff;
          const V3<R> ak = ld3<R>(s.ax + 3 * k);
          const V3<R> ok = ld3<R>(s.o + 3 * k);
          const bool rev = M.li[k * LI_COLS + LI_JTYPE] == J_REV;
          gv[k4] = rev ? dot(ak, add(Ua, cross(sub(oi, ok), Ul))) : dot(ak, Ul);
        }
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
          if (q0 + k4 < qe) s.G[q0 + k4] = gv[k4];
      }
    }
    // velocities under v*: roots at level 0, one-DOF joints below (operands read at once, no branch on the
    // joint type)
    for (int d = 0; d < M.n_levels; ++d) {
      for (int idx = M.level_begin[d] + tt; idx < M.level_begin[d + 1]; idx += TEAM) {
        const int i = M.level_links[idx];
        const int* li = M.li + i * LI_COLS;
        V3<R> w, vl;
        if (d == 0) {
          w = mk(R(0), R(0), R(0));
          vl = w;
          if (li[LI_JTYPE] == J_FREE) {
            const int c = li[LI_ROOTCOL];
            vl = ld3<R>(s.vs + c);
            w = ld3<R>(s.vs + c + 3);
          }
        } else {
          const int jt = li[LI_JTYPE], p = li[LI_PARENT], c = li[LI_COL];
          const V3<R> oi = ld3<R>(s.o + 3 * i), op = ld3<R>(s.o + 3 * p);
          const V3<R> wp = ld3<R>(s.v + 6 * p), vp = ld3<R>(s.v + 6 * p + 3);
          const V3<R> ax = ld3<R>(s.ax + 3 * i);
          const R qd = s.vs[c];
          w = wp;
          vl = add(vp, cross(wp, sub(oi, op)));
          if (jt == J_REV) w = add(w, mul(ax, qd));
          else vl = add(vl, mul(ax, qd));
        }
        st3(s.v + 6 * i, w);
        st3(s.v + 6 * i + 3, vl);
      }
      __syncthreads();
    }

    PHASE_MARK(5);
    // ---------------------------------------------------- narrow phase and activation (one slot per lane)
    for (int sb = 0; sb < ns; sb += TEAM) {
      const int sl = sb + tt;
      if (sl < ns) {
        const int* si = M.si + sl * SI_COLS;
        const double* sf = M.sf + sl * SF_COLS;
        const int ka = si[SI_LINK_A], kb = si[SI_LINK_B];
        const R rad = R(sf[SF_R]);
        R Ra[9];
        quat_R(s.q + 4 * ka, Ra);
        const V3<R> xc = add(ld3<R>(s.o + 3 * ka), mv(Ra, ld3<R>(sf + SF_P)));
        R phi;
        V3<R> nrm, x;
        if (si[SI_TYPE] == SLOT_SPHERE_PLANE) {
          phi = origin.z + xc.z - rad;
          nrm = mk(R(0), R(0), R(1));
          x = sub(xc, mk(R(0), R(0), rad));
        } else if (si[SI_TYPE] == SLOT_CORNER_PLANE) {
          phi = origin.z + xc.z;
          nrm = mk(R(0), R(0), R(1));
          x = xc;
        } else {
          // sphere against box: closest point, or the face of least penetration when inside
          R Rb[9];
          quat_R(s.q + 4 * kb, Rb);
          const V3<R> cb = add(ld3<R>(s.o + 3 * kb), mv(Rb, ld3<R>(sf + SF_BOXC)));
          const V3<R> hb = ld3<R>(sf + SF_HALF);
          const V3<R> xl = mtv(Rb, sub(xc, cb));
          const V3<R> ql = mk(min_(max_(xl.x, -hb.x), hb.x), min_(max_(xl.y, -hb.y), hb.y), min_(max_(xl.z, -hb.z), hb.z));
          const bool inside = ql.x == xl.x && ql.y == xl.y && ql.z == xl.z;
          const V3<R> dl = sub(xl, ql);
          const R dn = sqrt_(dot(dl, dl));
          V3<R> nl;
          if (!inside && dn > R(1e-12)) {
            phi = dn - rad;
            nl = mul(dl, R(1) / dn);
          } else {
            const R pen[3] = {hb.x - abs_(xl.x), hb.y - abs_(xl.y), hb.z - abs_(xl.z)};
            const R xs[3] = {xl.x, xl.y, xl.z};
            int kbest = 0;
            if (pen[1] < pen[kbest]) kbest = 1;
            if (pen[2] < pen[kbest]) kbest = 2;
            const R sg = xs[kbest] >= R(0) ? R(1) : R(-1);
            nl = kbest == 0 ? mk(sg, R(0), R(0)) : (kbest == 1 ? mk(R(0), sg, R(0)) : mk(R(0), R(0), sg));
            phi = -pen[kbest] - rad;
          }
          nrm = mv(Rb, nl);
          x = sub(xc, mul(nrm, rad));
        }
        // normal velocity of body a relative to body b at x under v*
        V3<R> ua = add(ld3<R>(s.v + 6 * ka + 3), cross(ld3<R>(s.v + 6 * ka), sub(x, ld3<R>(s.o + 3 * ka))));
        if (kb >= 0) ua = sub(ua, add(ld3<R>(s.v + 6 * kb + 3), cross(ld3<R>(s.v + 6 * kb), sub(x, ld3<R>(s.o + 3 * kb)))));
        const R vn = dot(nrm, ua);
        s.phi[sl] = phi;
        st3(s.n + 3 * sl, nrm);
        st3(s.x + 3 * sl, x);
        s.sact[sl] = (phi + h * min_(R(0), vn)) < R(P.mc);
      }
    }
    __syncthreads();

    PHASE_MARK(6);
    // ---------------------------------------------------- constraint rows: limits (by DOF), then contacts
    // row descriptor: kind << 16 | DOF (kinds 1, 2: lower, upper limit) or slot (3, 4, 5: normal, t1, t2);
    // the normal row of friction row r is r - (kind - 3)
    {
      int running = 0;
      for (int jb = 0; jb < nd; jb += TEAM) {
        const int j = jb + tt;
        int alo = 0, ahi = 0;
        R glo = R(0), ghi = R(0);
        if (j < nd) {
          const int lk = M.dof_link[j];
          const double* lf = M.lf + lk * LF_COLS;
          const R vs = s.vs[M.li[lk * LI_COLS + LI_COL]];
          const R ml = R(lf[LF_ML]), q = s.qj[j];
          const double lo = P.dof_limits ? double(P.dof_limits[2 * (dbase + j)]) : lf[LF_LO];
          const double hi = P.dof_limits ? double(P.dof_limits[2 * (dbase + j) + 1]) : lf[LF_HI];
          if (isfinite(lo)) {
            glo = q - R(lo);
            alo = min_(glo, glo + h * vs) < ml;
          }
          if (isfinite(hi)) {
            ghi = R(hi) - q;
            ahi = min_(ghi, ghi - h * vs) < ml;
          }
        }
        const unsigned long long mlo = team_ballot<TEAM>(tm, alo), mhi = team_ballot<TEAM>(tm, ahi);
        const int base = running + __popcll(mlo & lanes_below(tt)) + __popcll(mhi & lanes_below(tt));
        // rbias: the row's bias, or with the temporal solver its position error (the bias is then formed
        // before every sweep)
        if (alo) {
          s.rkr[base] = (1 << 16) | j;
          s.rbias[base] = tgs ? glo : row_bias(glo, h, R(P.beta));
        }
        if (ahi) {
          const int r = base + alo;
          s.rkr[r] = (2 << 16) | j;
          s.rbias[r] = tgs ? ghi : row_bias(ghi, h, R(P.beta));
        }
        running += __popcll(mlo) + __popcll(mhi);
      }
      for (int sb = 0; sb < ns; sb += TEAM) {
        const int sl = sb + tt;
        const int a = sl < ns ? s.sact[sl] : 0;
        const unsigned long long m = team_ballot<TEAM>(tm, a);
        const int base = running + 3 * __popcll(m & lanes_below(tt));
        if (sl < ns) s.sact[sl] = a ? base : -1;  // from here on: the slot's first row
        if (a) {
          const R phi = s.phi[sl];
          for (int k = 0; k < 3; ++k) {
            s.rkr[base + k] = ((3 + k) << 16) | sl;
            s.rbias[base + k] = k == 0 ? (tgs ? phi : row_bias(phi, h, R(P.beta))) : R(0);
          }
        }
        running += 3 * __popcll(m);
      }
      if (tt == 0) s.misc[0] = running;
    }
    __syncthreads();
    const int Rn = s.misc[0];
    // largest row count of the wavefront's teams (uniform; read while every lane is active)
    int rn_w = Rn;
#pragma unroll
    for (int q = 1; q < EPW; ++q) rn_w = max(rn_w, lane_read(Rn, q * TEAM));
    rn_w = lane_read(rn_w, 0);

    PHASE_MARK(7);
    // ---------------------------------------------------- row Jacobians and responses W_r = M~^-1 J_r^T
    // Up to FR rows (one per lane) keep their Jacobian in registers (compact form) and W in LDS and are
    // solved in registers below; more rows (or rows too long for the compact form) go through global scratch.
    const bool fast = Rn <= FR && M.jfast;
    // more rows than one chunk but no more than the lanes of the environment: every lane keeps its own row's
    // compact Jacobian (lane k: row k), the responses still go in chunks of FR rows, and Gauss-Seidel runs
    // in the Delassus form with the columns of A streamed from global scratch instead of held in registers
    const bool wide = !fast && TEAM == 64 && M.jfast && Rn <= TEAM;
    slow_any = slow_any || !fast;
    rows_max = max(rows_max, Rn);
    if (!fast && !wide)
      for (int k = tt; k < Rn * nv; k += TEAM) Jg[k] = R(0);
    JRow<R> jr;  // fast and wide paths: this lane's row
    jrow_clear(jr);
    if (wide && tt >= FR && tt < Rn) {  // rows past the first chunk: their lanes form the compact row here
      const int kr = s.rkr[tt];
      const int kind = kr >> 16, ref = kr & 0xffff;
      if (kind <= 2) {
        jr.c[0] = M.li[M.dof_link[ref] * LI_COLS + LI_COL];
        jr.val[0] = kind == 1 ? R(1) : R(-1);
      } else {
        V3<R> dd = ld3<R>(s.n + 3 * ref);
        if (kind != 3) {
          V3<R> t1, t2;
          tangents(dd, t1, t2);
          dd = kind == 4 ? t1 : t2;
        }
        jrow_point(M, s, M.si[ref * SI_COLS + SI_LINK_A], M.si[ref * SI_COLS + SI_LINK_B], ld3<R>(s.x + 3 * ref), dd,
                   jr);
      }
    }
    __syncthreads();
    for (int rb = 0; rb < Rn; rb += FR) {  // chunks of FR rows, one per lane
      // the lanes of this chunk form their compact rows (fast path, and the first chunk of the wide path)
      const bool jreg = fast || (wide && rb == 0);
      const int r = tt < FR ? rb + tt : Rn;
      const auto Wrow = s.W + tt * L.wstride;  // only lanes tt < FR own a row of the block
      R* const JrowG = Jg + (long long)r * nv;
      if (tt < FR)
        for (int c = 0; c < nv; ++c) Wrow[c] = R(0);
      if (r < Rn) {
        const int kr = s.rkr[r];
        const int kind = kr >> 16, ref = kr & 0xffff;
        int lk = 0, ka = 0, kb = -1;
        R sg = R(0);
        V3<R> dd = mk(R(0), R(0), R(0)), x = dd;
        if (kind <= 2) {
          lk = M.dof_link[ref];
          sg = kind == 1 ? R(1) : R(-1);
          const int col = M.li[lk * LI_COLS + LI_COL];
          if (jreg) {
            jr.c[0] = col;
            jr.val[0] = sg;
          } else if (!wide) {
            JrowG[col] = sg;
          }
          unit_load_inward(M, s, lk, mk(R(0), R(0), R(0)), mk(R(0), R(0), R(0)), sg, Wrow);
        } else {
          const V3<R> nrm = ld3<R>(s.n + 3 * ref);
          dd = nrm;
          if (kind != 3) {
            V3<R> t1, t2;
            tangents(nrm, t1, t2);
            dd = kind == 4 ? t1 : t2;
          }
          x = ld3<R>(s.x + 3 * ref);
          ka = M.si[ref * SI_COLS + SI_LINK_A];
          kb = M.si[ref * SI_COLS + SI_LINK_B];
          unit_load_inward(M, s, ka, mul(cross(sub(x, ld3<R>(s.o + 3 * ka)), dd), R(-1)), mul(dd, R(-1)), R(0), Wrow);
          if (kb >= 0) unit_load_inward(M, s, kb, cross(sub(x, ld3<R>(s.o + 3 * kb)), dd), dd, R(0), Wrow);
          if (jreg) {
            jrow_point(M, s, ka, kb, x, dd, jr);
          } else if (!wide) {
            point_row(M, s, ka, x, dd, R(1), JrowG, Wrow, true, false);
            if (kb >= 0) point_row(M, s, kb, x, dd, R(-1), JrowG, Wrow, true, false);
          }
        }
        // roots: a = -(I^A_root)^-1 (accumulated bias force); generalized root columns are (v_com, w)
        for (int k = 0; k < na; ++k) {
          const int* ai = M.ai + k * AI_COLS;
          if (ai[AI_FIXED]) continue;
          const int c = ai[AI_COL];
          R x6[6];
#pragma unroll
          for (int q = 0; q < 6; ++q) x6[q] = -Wrow[c + q];
          chol6_solve(s.L0 + 27 * k, s.L0 + 27 * k + 21, x6);
          Wrow[c + 0] = x6[3]; Wrow[c + 1] = x6[4]; Wrow[c + 2] = x6[5];
          Wrow[c + 3] = x6[0]; Wrow[c + 4] = x6[1]; Wrow[c + 5] = x6[2];
        }
      }
      __syncthreads();
      // outward: qdd_i = (u_i - Ubar_i . a_root - sum_k G_ik qdd_k) / D_i, level by level with lanes over the
      // (row, link) pairs of a level, so that the chain has one step per tree level instead of one per link
      {
        const int rows_here = min(FR, max(0, Rn - rb));
        for (int d = 1; d < M.n_levels; ++d) {
          const int b = M.level_begin[d], n_at = M.level_begin[d + 1] - b;
          const int pairs = rows_here * n_at;
          const float inv_at = __builtin_amdgcn_rcpf(float(n_at));  // within an ulp: the rounding below has margin
          for (int pi = tt; pi < pairs; pi += TEAM) {
            // row and link of the pair without an integer division ((pi + 1/2) / n_at is at least 1/(2 n_at) from
            // an integer, far above the rounding of the product for pi < 2^16)
            const int q_ = int((float(pi) + 0.5f) * inv_at);
            const int i = M.level_links[b + pi - q_ * n_at];
            // the link's record, then every operand read before the arithmetic and no branch on the link
            // (past level 0 every link has a one-DOF joint; entries past the last ancestor read the last one
            // again and add zero)
            const int* li = M.li + i * LI_COLS;
            const int rc = li[LI_ROOTCOL], qb = li[LI_ANC_BEGIN], qe = li[LI_ANC_END], c = li[LI_COL];
            const auto Wq = s.W + q_ * L.wstride;
            const int rcs = max(rc, 0);
            const V3<R> ub = ld3<R>(s.Ubar + 3 * i), ul = ld3<R>(s.U + 6 * i + 3);
            const R w0 = Wq[rcs + 0], w1 = Wq[rcs + 1], w2 = Wq[rcs + 2], w3 = Wq[rcs + 3], w4 = Wq[rcs + 4],
                    w5 = Wq[rcs + 5];
            const R wc = Wq[c], dinv = s.Dinv[i];
            R acc = rc >= 0 ? ub.x * w3 + ub.y * w4 + ub.z * w5 + ul.x * w0 + ul.y * w1 + ul.z * w2 : R(0);
            for (int q0 = qb; q0 < qe; q0 += 8) {
              R g[8], wv[8];
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const int q = min(q0 + k, qe - 1);
                g[k] = s.G[q];
                wv[k] = Wq[M.anc_link[q] >> 16];
              }
#pragma unroll
              for (int k = 0; k < 8; ++k) acc += (q0 + k < qe ? g[k] : R(0)) * wv[k];
            }
            Wq[c] = (wc - acc) * dinv;
          }
          __syncthreads();
        }
      }
      if (r < Rn) {
        // A_rr = J_r W_r (the slow path re-derives its row's direction and point from the row tables)
        R A;
        if (jreg) {
          A = jrow_dot(jr, Wrow);
        } else {
          const int kr = s.rkr[r];
          const int kind = kr >> 16, ref = kr & 0xffff;
          if (kind <= 2) {
            A = (kind == 1 ? R(1) : R(-1)) * Wrow[M.li[M.dof_link[ref] * LI_COLS + LI_COL]];
          } else {
            V3<R> dd = ld3<R>(s.n + 3 * ref);
            if (kind != 3) {
              V3<R> t1, t2;
              tangents(dd, t1, t2);
              dd = kind == 4 ? t1 : t2;
            }
            const V3<R> x = ld3<R>(s.x + 3 * ref);
            const int ka = M.si[ref * SI_COLS + SI_LINK_A], kb = M.si[ref * SI_COLS + SI_LINK_B];
            A = point_row(M, s, ka, x, dd, R(1), Wrow, Wrow, false, true);
            if (kb >= 0) A += point_row(M, s, kb, x, dd, R(-1), Wrow, Wrow, false, true);
          }
        }
        s.rinvA[r] = A >= R(kMinRowMass) ? R(1) / A : R(0);
        s.rlam[r] = R(0);
      }
      __syncthreads();
      if (wide) {
        // column block of A: lane k forms A[k][r] = J_k W_r for this chunk's rows (A_rk in the column of row r,
        // A being symmetric), and its own row's 1/A_kk from the same product
        const int rows_here = min(FR, Rn - rb);
        R diag = R(0);
        if (tt < Rn)
          for (int q = 0; q < rows_here; ++q) {
            const R a = jrow_dot(jr, s.W + q * L.wstride);
            Ag[(long long)(rb + q) * TEAM + tt] = a;
            diag = rb + q == tt ? a : diag;
          }
        if (tt >= rb && tt < rb + rows_here) s.rinvA[tt] = diag >= R(kMinRowMass) ? R(1) / diag : R(0);
      }
      if (!fast) {
        const int rows_here = min(FR, Rn - rb);
        for (int q = 0; q < rows_here; ++q)
          for (int c = tt; c < nv; c += TEAM) Wg[(long long)(rb + q) * nv + c] = s.W[q * L.wstride + c];
        __syncthreads();
      }
    }
    for (int r = tt; r < Rn; r += TEAM) {  // friction rows of a dropped normal row are dropped too
      const int kind = s.rkr[r] >> 16;
      if (kind >= 4 && s.rinvA[r - (kind - 3)] == R(0)) s.rinvA[r] = R(0);
    }
    __syncthreads();

    PHASE_MARK(8);
    // ---------------------------------------------------- projected Gauss-Seidel
    const R mu = R(P.env_mu ? double(P.env_mu[env]) : P.mu);
    R vj;
    if (fast) {
      // Delassus form, one row per lane: lane k holds y_k = J_k v and column k of A = J M~^-1 J^T
      // (Acol[r] = J_k W_r, A being symmetric).  The wavefront runs the rows of its teams in lockstep, up to
      // the larger row count rn_w.
      R Acol[FR];  // rows r >= this team's count have W_r = 0
#pragma unroll
      for (int r = 0; r < FR; ++r) Acol[r] = r < rn_w ? jrow_dot(jr, s.W + r * L.wstride) : R(0);
      R y = jrow_dot(jr, s.vs);
      const bool own = tt < Rn;
      const R ia = own ? s.rinvA[tt] : R(0);
      const int kindv = own ? (s.rkr[tt] >> 16) : 0;
      const bool fric = kindv >= 4;
      const int nrmv = fric ? tt - (kindv - 3) : -1;
      // temporal solver: pos is the row's position error, advanced by h / iters J_k v after every sweep
      R pos = own && tgs ? s.rbias[tt] : R(0);
      R bias = own ? (tgs ? (fric ? R(0) : row_bias(pos, h, R(P.beta))) : s.rbias[tt]) : R(0);
      // every lane evaluates the update of its own row; the one of row r is applied and its impulse change
      // broadcast.  A friction lane follows its normal row's impulse through those broadcasts and keeps its
      // box bounds +-mu lambda_n.  Rows without a response (1/A_rr = 0: dropped, or lanes past the row count)
      // hold lambda = 0 and their update is a clamp of 0, so they need no test.  c = lambda - b / A_rr.
      // The bounds are updated by arithmetic on every row (hi += mu dl with dl zero unless the broadcast row
      // is the lane's normal row; lo = -hi for friction rows, -0 for the others, whose upper bound is a
      // finite stand-in for infinity): values that come out of arithmetic need no canonicalizing before the
      // clamp, and no selects are needed.
      const R fsign = fric ? R(1) : R(0);
      R lam = R(0), hi = fric ? R(0) : R(kOpenBound), lo = R(0), bia = bias * ia;
      R c = -bia;
      const R hstep = h / R(max(P.iters, 1));
      for (int it = 0; it < P.iters; ++it) {
        if (tgs && it > 0 && own && !fric) {
          bias = row_bias(pos, h, R(P.beta));
          bia = bias * ia;
          c = lam - bia;
        }
        // opaque copies of the lane's row and normal-row indices and of the row count: keeps the per-row
        // compares inside the sweep instead of 3 x FR hoisted (and spilled) masks
        int me = tt, mn = nrmv, rw = rn_w;
        R muv = mu;  // in a vector register: a spilled scalar copy would be reloaded at every row
        asm volatile("" : "+v"(me), "+v"(mn), "+s"(rw), "+v"(muv));
#pragma unroll
        for (int r = 0; r < FR; ++r) {
          if (r < rw) {
            const R cand = clamp_(fma_(-y, ia, c), lo, hi);
            const R dl = team_read<TEAM>(tm, cand - lam, r);
            lam = me == r ? cand : lam;
            c = lam - bia;
            hi = fma_(mn == r ? muv : R(0), dl, hi);
            lo = -(hi * fsign);
            y += Acol[r] * dl;
          }
        }
        if (tgs) pos += hstep * y;  // y = J_k v at the end of the sweep
      }
      if (own) s.rlam[tt] = lam;
      __syncthreads();
      // v+ = v* + sum_r W_r lambda_r, lanes over velocity columns
      vj = tt < nv ? s.vs[tt] : R(0);
      if (tt < nv)
        for (int r = 0; r < Rn; ++r) vj += s.rlam[r] * s.W[r * L.wstride + tt];
    } else if (wide) {
      // the register form above with up to TEAM rows: lane k holds y_k = J_k v and reads A[k][r] from the column
      // of row r in global scratch, kWideAhead rows ahead of the update that uses it
      R y = tt < Rn ? jrow_dot(jr, s.vs) : R(0);
      const bool own = tt < Rn;
      const R ia = own ? s.rinvA[tt] : R(0);
      const int kindv = own ? (s.rkr[tt] >> 16) : 0;
      const bool fric = kindv >= 4;
      const int nrmv = fric ? tt - (kindv - 3) : -1;
      R pos = own && tgs ? s.rbias[tt] : R(0);
      R bias = own ? (tgs ? (fric ? R(0) : row_bias(pos, h, R(P.beta))) : s.rbias[tt]) : R(0);
      const R fsign = fric ? R(1) : R(0);
      R lam = R(0), hi = fric ? R(0) : R(kOpenBound), lo = R(0), bia = bias * ia;
      R c = -bia;
      const R hstep = h / R(max(P.iters, 1));
      const R* const acol = Ag + tt;
      for (int it = 0; it < P.iters; ++it) {
        if (tgs && it > 0 && own && !fric) {
          bias = row_bias(pos, h, R(P.beta));
          bia = bias * ia;
          c = lam - bia;
        }
        R nx[kWideAhead];
#pragma unroll
        for (int q = 0; q < kWideAhead; ++q) nx[q] = own && q < Rn ? acol[q * TEAM] : R(0);
        for (int r0 = 0; r0 < Rn; r0 += kWideAhead) {
          R cur[kWideAhead];
#pragma unroll
          for (int q = 0; q < kWideAhead; ++q) {
            cur[q] = nx[q];
            const int rn = r0 + kWideAhead + q;
            nx[q] = own && rn < Rn ? acol[rn * TEAM] : R(0);  // lanes without a row read nothing
          }
#pragma unroll
          for (int q = 0; q < kWideAhead; ++q) {
            const int r = r0 + q;
            if (r < Rn) {
              const R cand = clamp_(fma_(-y, ia, c), lo, hi);
              const R dl = team_read<TEAM>(tm, cand - lam, r);
              lam = tt == r ? cand : lam;
              c = lam - bia;
              hi = fma_(nrmv == r ? mu : R(0), dl, hi);
              lo = -(hi * fsign);
              y += cur[q] * dl;
            }
          }
        }
        if (tgs) pos += hstep * y;
      }
      if (own) s.rlam[tt] = lam;
      __syncthreads();
      vj = tt < nv ? s.vs[tt] : R(0);
      if (tt < nv)
        for (int r = 0; r < Rn; ++r) vj += s.rlam[r] * Wg[(long long)r * nv + tt];
    } else {
      // lanes over velocity columns, rows streamed from global scratch
      vj = tt < nv ? s.vs[tt] : R(0);
      const R hstep = h / R(max(P.iters, 1));
      for (int it = 0; it < P.iters; ++it) {
        for (int r = 0; r < Rn; ++r) {
          const R invA = s.rinvA[r];
          if (invA == R(0)) continue;
          const R Jr = tt < nv ? Jg[(long long)r * nv + tt] : R(0);
          const R Wr = tt < nv ? Wg[(long long)r * nv + tt] : R(0);
          const int kind = s.rkr[r] >> 16;
          // temporal solver: rbias holds the position error of limit and normal rows
          const R b = tgs ? (kind >= 4 ? R(0) : row_bias(s.rbias[r], h, R(P.beta))) : s.rbias[r];
          const R res = team_sum<TEAM>(Jr * vj) + b;
          const R lam = s.rlam[r];
          R nlam = lam - res * invA;
          if (kind >= 4) {
            const R hi = mu * s.rlam[r - (kind - 3)];
            nlam = min_(max_(nlam, -hi), hi);
          } else {
            nlam = max_(nlam, R(0));
          }
          vj += Wr * (nlam - lam);
          s.rlam[r] = nlam;
        }
        if (tgs) {  // advance the position errors by h / iters J_r v
          for (int r = 0; r < Rn; ++r) {
            const int kind = s.rkr[r] >> 16;
            if (s.rinvA[r] == R(0) || kind >= 4) continue;
            const R Jr = tt < nv ? Jg[(long long)r * nv + tt] : R(0);
            const R nb = s.rbias[r] + hstep * team_sum<TEAM>(Jr * vj);
            s.rbias[r] = nb;  // every lane of the team writes the same value
          }
        }
      }
    }
    __syncthreads();

    PHASE_MARK(9);
    // ---------------------------------------------------- outputs of the substep and integration
    if (P.dbg_rc && valid) {
      int running = 0;
      for (int rb = 0; rb < Rn; rb += TEAM) {
        const int r = rb + tt;
        const int keep = r < Rn && s.rinvA[r] != R(0);
        const unsigned long long m = team_ballot<TEAM>(tm, keep);
        const int pos = running + __popcll(m & lanes_below(tt));
        if (keep && pos < M.r_cap) {
          const int kr = s.rkr[r];
          const int kind = kr >> 16, ref = kr & 0xffff;
          const long long o = (long long)env * P.dbg_row_stride + (long long)sub_i * P.dbg_row_sub + pos;
          P.dbg_key[o] = kind <= 2 ? (kind << 24) | (ref << 8) : (kind << 24) | M.si[ref * SI_COLS + SI_KEY];
          P.dbg_lam[o] = float(s.rlam[r]);
        }
        running += __popcll(m);
      }
      if (tt == 0) P.dbg_rc[env * P.substeps + sub_i] = running;
    }
    // contact impulses of each slot -> force on its bodies (summed over the step, divided by dt)
    for (int sb = 0; sb < ns; sb += TEAM) {
      const int sl = sb + tt;
      if (sl < ns) {
        const int r = s.sact[sl];
        V3<R> F = mk(R(0), R(0), R(0));
        if (r >= 0) {
          const V3<R> nrm = ld3<R>(s.n + 3 * sl);
          V3<R> t1, t2;
          tangents(nrm, t1, t2);
          F = add(add(mul(nrm, s.rlam[r]), mul(t1, s.rlam[r + 1])), mul(t2, s.rlam[r + 2]));
        }
        st3(s.x + 3 * sl, F);  // the contact point is no longer needed
      }
    }
    __syncthreads();
    for (int b = tt; b < nl; b += TEAM) {
      V3<R> acc = ld3<R>(s.F_ + 3 * b);
      for (int q = M.body_slot_begin[b]; q < M.body_slot_begin[b + 1]; ++q) {
        const int e = M.body_slot[q];
        const V3<R> F = ld3<R>(s.x + 3 * (e >> 1));
        acc = (e & 1) ? sub(acc, F) : add(acc, F);
      }
      st3(s.F_ + 3 * b, acc);
    }
    // DOF forces at the end-of-substep velocity, and joint integration q+ = q + h qd+
    if (tt < nv) s.qd[tt] = vj;
    __syncthreads();
    for (int j = tt; j < nd; j += TEAM) {
      const int lk = M.dof_link[j];
      const double* lf = M.lf + lk * LF_COLS;
      const int c = M.li[lk * LI_COLS + LI_COL];
      const R pt = P.pos_tgt ? R(P.pos_tgt[dbase + j]) : R(0);
      const R vt = P.vel_tgt ? R(P.vel_tgt[dbase + j]) : R(0);
      const R qdp = s.qd[c];
      const R kp = R(P.dof_kp ? double(P.dof_kp[dbase + j]) : lf[LF_KP]);
      const R kd = R(P.dof_kd ? double(P.dof_kd[dbase + j]) : lf[LF_KD]);
      dof_force_acc += R(P.act[dbase + j]) + kp * (pt - s.qj[j] - h * qdp) + kd * (vt - qdp);
      s.qj[j] += h * qdp;
    }
    // free roots: p+ = p + h v+, quat+ = normalize(Exp(h w+) (x) quat)
    for (int k = tt; k < na; k += TEAM) {
      const int* ai = M.ai + k * AI_COLS;
      if (ai[AI_FIXED]) continue;
      const int c = ai[AI_COL];
      const auto rs = s.root + 13 * k;
      const V3<R> vc = ld3<R>(s.qd + c), w = ld3<R>(s.qd + c + 3);
      st3(rs, add(ld3<R>(rs), mul(vc, h)));
      const V3<R> th = mul(w, h);
      const R ang = sqrt_(dot(th, th));
      R dx, dy, dz, dw;
      if (ang < R(1e-8)) {
        dx = R(0.5) * th.x; dy = R(0.5) * th.y; dz = R(0.5) * th.z; dw = R(1);
      } else {
        R sn, cs;
        sincos_(R(0.5) * ang, &sn, &cs);
        const R sc = sn / ang;
        dx = th.x * sc; dy = th.y * sc; dz = th.z * sc; dw = cs;
      }
      const R qx = rs[3], qy = rs[4], qz = rs[5], qw = rs[6];
      // Hamilton product (dx, dy, dz, dw) (x) (qx, qy, qz, qw)
      const R nx = dw * qx + qw * dx + (dy * qz - dz * qy);
      const R ny = dw * qy + qw * dy + (dz * qx - dx * qz);
      const R nz = dw * qz + qw * dz + (dx * qy - dy * qx);
      const R nw = dw * qw - (dx * qx + dy * qy + dz * qz);
      const R inv = rsqrt_(nx * nx + ny * ny + nz * nz + nw * nw);
      rs[3] = nx * inv; rs[4] = ny * inv; rs[5] = nz * inv; rs[6] = nw * inv;
      st3(rs + 7, vc);
      st3(rs + 10, w);
    }
    __syncthreads();
    if (P.mid_root && sub_i + 1 < P.substeps && valid) {  // state after this substep, for the adjoint
      double* mr = P.mid_root + (long long)sub_i * P.mid_block + (long long)abase * 13;
      double* md = P.mid_dof + (long long)sub_i * P.mid_block + (long long)dbase * 2;
      for (int k = tt; k < 13 * na; k += TEAM) mr[k] = double(s.root[k]);
      for (int j = tt; j < nd; j += TEAM) {
        md[2 * j] = double(s.qj[j]);
        md[2 * j + 1] = double(s.qd[M.li[M.dof_link[j] * LI_COLS + LI_COL]]);
      }
    }
    PHASE_MARK(-1);
  }

  // ---------------------------------------------------------------- rigid-body states of the new state
  if (P.rb_state) {
    stage_joint_locals<R, EPW, TEAM>(M, s, tt);
    __syncthreads();
    for (int d = 0; d < M.n_levels; ++d) {
      for (int idx = M.level_begin[d] + tt; idx < M.level_begin[d + 1]; idx += TEAM) {
        const int i = M.level_links[idx];
        R Rw[9], qq[4];
        V3<R> o, w, vl, ax;
        link_kinematics(M, s, i, origin, Rw, qq, o, w, vl, ax, d == 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) s.q[4 * i + k] = qq[k];
        st3(s.o + 3 * i, o);
        st3(s.v + 6 * i, w);
        st3(s.v + 6 * i + 3, vl);
        if (valid) {
          float* dst = P.rb_state + (long long)(bbase + i) * 13;
          const V3<R> x = add(o, origin);
          dst[0] = float(x.x); dst[1] = float(x.y); dst[2] = float(x.z);
#pragma unroll
          for (int k = 0; k < 4; ++k) dst[3 + k] = float(qq[k]);
          dst[7] = float(vl.x); dst[8] = float(vl.y); dst[9] = float(vl.z);
          dst[10] = float(w.x); dst[11] = float(w.y); dst[12] = float(w.z);
        }
      }
      __syncthreads();
    }
  }

  // ---------------------------------------------------------------- status word
  // bit 0: the new state is not finite; bit 1: a substep took the row-response slow path
  if (P.env_status) {
    int bad = 0;
    for (int k = tt; k < 13 * na; k += TEAM) bad |= !isfinite(s.root[k]);
    for (int j = tt; j < nd; j += TEAM) bad |= !isfinite(s.qj[j]);
    for (int c = tt; c < nv; c += TEAM) bad |= !isfinite(s.qd[c]);
    const unsigned long long m = team_ballot<TEAM>(tm, bad);
    if (valid && tt == 0) P.env_status[env] = (m != 0ull ? 1 : 0) | (slow_any ? 2 : 0);
  }

  if (P.big_rows && valid && tt == 0) P.big_rows[env] = rows_max > kAdjBigRowsAt ? 1 : 0;
  if (P.env_rows && valid && tt == 0) P.env_rows[env] = rows_max;

  // ---------------------------------------------------------------- write back
  if (!valid) return;
  for (int k = tt; k < na; k += TEAM) {
    const int* ai = M.ai + k * AI_COLS;
    float* dst = P.root_state + (long long)(abase + k) * 13;
    for (int q = 0; q < 7; ++q) dst[q] = float(s.root[13 * k + q]);
    for (int q = 7; q < 13; ++q) dst[q] = ai[AI_FIXED] ? 0.0f : float(s.root[13 * k + q]);
  }
  for (int j = tt; j < nd; j += TEAM) {
    const int lk = M.dof_link[j];
    P.dof_state[2ll * (dbase + j)] = float(s.qj[j]);
    P.dof_state[2ll * (dbase + j) + 1] = float(s.qd[M.li[lk * LI_COLS + LI_COL]]);
    if (P.dof_force) P.dof_force[dbase + j] = float(dof_force_acc / R(P.substeps));
  }
  if (CYC && P.dbg_cycles && tt == 0)
    for (int k = 0; k < kPhases; ++k) P.dbg_cycles[(long long)env * kPhases + k] = cyc[k];
#undef PHASE_MARK
  if (P.contact_force) {
    const R inv_dt = R(1) / R(P.dt);
    for (int k = tt; k < 3 * nl; k += TEAM) P.contact_force[(long long)bbase * 3 + k] = float(s.F_[k] * inv_dt);
  }
}

// Register budget: two wavefronts per SIMD (<= 256 VGPRs) so that one hides the other's latency, except
// for the FP64 two-environments-per-wavefront form whose LDS allows one workgroup per SIMD anyway.
template <typename R, int TEAM>
constexpr int kWavesPerEU = (sizeof(R) == 4 || TEAM == 64) ? 2 : 1;
// the per-type FP32 launch with one env per wavefront fits three wavefronts per SIMD (<= 168 registers; its
// ~9 KB of LDS admits twelve workgroups per CU)
template <typename R, int TEAM>
constexpr int kStepWavesPerEU = (sizeof(R) == 4 && TEAM == 64) ? 3 : kWavesPerEU<R, TEAM>;

template <typename R, int TEAM, bool TGS, bool CYC = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kStepWavesPerEU<R, TEAM>))) void step_kernel(StepArgs P) {
  step_group<R, TEAM, TGS, CYC>(P, P.ty, blockIdx.x, true);
}

// persistent form: each workgroup walks the work list with a grid stride; the list is ordered by
// estimated cost, so the heaviest groups start first and the tail is made of the cheapest ones
template <typename R, int TEAM, bool TGS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<R, TEAM>))) void step_fused(FusedArgs A) {
  int prev = -1;
  for (int u = blockIdx.x; u < A.n_units; u += gridDim.x) {
    const int ty = A.units[2 * u], grp = A.units[2 * u + 1];
    __syncthreads();
    step_group<R, TEAM, TGS, false>(A.base, A.types[ty], grp, ty != prev);
    prev = ty;
  }
}

// Copy the rows of the listed actors from src to dst (same layout).  table holds 4 ints per actor:
// root row, root row count (1), first DOF row, DOF row count; `field` selects the pair (0 root, 2 DOF).
__global__ void set_rows_kernel(float* dst, const float* src, const int* idx, int n, int n_actors, const int* table,
                                int field, int width) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)n * kTeam) return;
  const int k = (int)(gid / kTeam), lane = (int)(gid % kTeam);
  const int a = idx ? idx[k] : k;
  if (a < 0 || a >= n_actors) return;  // invalid indices are ignored
  const int rb = table[4 * a + field], rc = table[4 * a + field + 1];
  for (int e = lane; e < rc * width; e += kTeam) {
    const long long off = (long long)rb * width + e;
    dst[off] = src[off];
  }
}

__global__ void scale_by_kp_kernel(float* x, const float* kp, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= kp[i];
}

template <typename R, int TEAM>
static hipError_t launch_one(const StepArgs& a, int n_envs, hipStream_t stream) {
  constexpr int EPW = kTeam / TEAM;
  const size_t lds = (size_t)a.ty.lds.total * sizeof(R);
  const int grid = (n_envs + EPW - 1) / EPW;
  if (a.dbg_cycles) {  // the instrumented instantiation (per-phase clock counters)
    if (a.solver == 1) hipLaunchKernelGGL((step_kernel<R, TEAM, true, true>), dim3(grid), dim3(kTeam), lds, stream, a);
    else hipLaunchKernelGGL((step_kernel<R, TEAM, false, true>), dim3(grid), dim3(kTeam), lds, stream, a);
  } else if (a.solver == 1) {
    hipLaunchKernelGGL((step_kernel<R, TEAM, true>), dim3(grid), dim3(kTeam), lds, stream, a);
  } else {
    hipLaunchKernelGGL((step_kernel<R, TEAM, false>), dim3(grid), dim3(kTeam), lds, stream, a);
  }
  return hipGetLastError();
}

template <typename R, int TEAM, bool TGS>
static const void* fused_fn() {
  return (const void*)step_fused<R, TEAM, TGS>;
}
template <bool TGS>
static const void* fused_kernel(int fp64, int team) {
  return fp64 ? (team == 32 ? fused_fn<double, 32, TGS>() : fused_fn<double, 64, TGS>())
              : (team == 32 ? fused_fn<float, 32, TGS>() : fused_fn<float, 64, TGS>());
}
template <bool TGS, bool CYC = false>
static const void* step_fn(int fp64, int team) {
  return fp64 ? (team == 32 ? (const void*)step_kernel<double, 32, TGS, CYC> : (const void*)step_kernel<double, 64, TGS, CYC>)
              : (team == 32 ? (const void*)step_kernel<float, 32, TGS, CYC> : (const void*)step_kernel<float, 64, TGS, CYC>);
}

// Counting sort of the env ids of one type by the rows of their last step, most rows first (rows of
// kOrderBuckets - 1 or more share the first bucket).  One workgroup; each thread keeps the ids and buckets
// of its kOrderPer entries in registers between the count and the scatter, and batches of up to
// kOrderLds ids are placed in LDS before one coalesced write (larger batches go through tmp).  The order
// within a bucket is whichever the LDS atomics give, which no result depends on.
constexpr int kOrderBuckets = 128;
constexpr int kOrderThreads = 1024;
constexpr int kOrderPer = 8;
constexpr int kOrderLds = kOrderThreads * kOrderPer;
__global__ __launch_bounds__(kOrderThreads) void order_by_rows_kernel(int* order, int* tmp, const int* rows, int n) {
  __shared__ int start[kOrderBuckets];
  __shared__ int placed[kOrderLds];
  const int t = threadIdx.x;
  const bool in_lds = n <= kOrderLds;
  auto bucket = [&](int e) { return kOrderBuckets - 1 - min(max(rows[e], 0), kOrderBuckets - 1); };
  if (t < kOrderBuckets) start[t] = 0;
  __syncthreads();
  int ids[kOrderPer], bk[kOrderPer];
#pragma unroll
  for (int k = 0; k < kOrderPer; ++k) {
    const int i = t + k * kOrderThreads;
    ids[k] = i < n ? order[i] : 0;
    bk[k] = i < n ? bucket(ids[k]) : 0;
  }
#pragma unroll
  for (int k = 0; k < kOrderPer; ++k)
    if (t + k * kOrderThreads < n) atomicAdd(&start[bk[k]], 1);
  for (int i = t + kOrderLds; i < n; i += kOrderThreads) atomicAdd(&start[bucket(order[i])], 1);
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int b = 0; b < kOrderBuckets; ++b) {
      const int c = start[b];
      start[b] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kOrderPer; ++k) {
    if (t + k * kOrderThreads < n) {
      const int pos = atomicAdd(&start[bk[k]], 1);
      if (in_lds) placed[pos] = ids[k];
      else tmp[pos] = ids[k];
    }
  }
  for (int i = t + kOrderLds; i < n; i += kOrderThreads) {
    const int e = order[i];
    tmp[atomicAdd(&start[bucket(e)], 1)] = e;
  }
  __syncthreads();
  if (in_lds)
    for (int i = t; i < n; i += kOrderThreads) order[i] = placed[i];
  else
    for (int i = t; i < n; i += kOrderThreads) order[i] = tmp[i];
}

hipError_t launch_order_by_rows(int* order, int* tmp, const int* rows, int n, hipStream_t stream) {
  if (n <= 1) return hipSuccess;
  hipLaunchKernelGGL(order_by_rows_kernel, dim3(1), dim3(kOrderThreads), 0, stream, order, tmp, rows, n);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int n_envs, int fp64, int team, hipStream_t stream) {
  if (n_envs <= 0) return hipSuccess;
  if (fp64) return team == 32 ? launch_one<double, 32>(a, n_envs, stream) : launch_one<double, 64>(a, n_envs, stream);
  return team == 32 ? launch_one<float, 32>(a, n_envs, stream) : launch_one<float, 64>(a, n_envs, stream);
}

hipError_t launch_scale_by_kp(float* x, const float* kp, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_by_kp_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, x, kp, n);
  return hipGetLastError();
}

template <bool TGS>
static void launch_fused_solver(const FusedArgs& a, int grid, size_t lds_bytes, int fp64, int team, hipStream_t stream) {
  if (fp64) {
    if (team == 32) hipLaunchKernelGGL((step_fused<double, 32, TGS>), dim3(grid), dim3(kTeam), lds_bytes, stream, a);
    else hipLaunchKernelGGL((step_fused<double, 64, TGS>), dim3(grid), dim3(kTeam), lds_bytes, stream, a);
  } else {
    if (team == 32) hipLaunchKernelGGL((step_fused<float, 32, TGS>), dim3(grid), dim3(kTeam), lds_bytes, stream, a);
    else hipLaunchKernelGGL((step_fused<float, 64, TGS>), dim3(grid), dim3(kTeam), lds_bytes, stream, a);
  }
}

hipError_t launch_step_fused(const FusedArgs& a, int grid, size_t lds_bytes, int fp64, int team, hipStream_t stream) {
  if (a.n_units <= 0) return hipSuccess;
  if (a.base.solver == 1) launch_fused_solver<true>(a, grid, lds_bytes, fp64, team, stream);
  else launch_fused_solver<false>(a, grid, lds_bytes, fp64, team, stream);
  return hipGetLastError();
}

hipError_t set_fused_lds_limit(int fp64, int team, size_t bytes) {
  hipError_t e = hipFuncSetAttribute(fused_kernel<false>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute(fused_kernel<true>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

hipError_t fused_blocks_per_cu(int fp64, int team, size_t lds_bytes, int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fused_kernel<false>(fp64, team), kTeam, lds_bytes);
}

hipError_t set_lds_limit(int fp64, int team, size_t bytes) {
  hipError_t e = hipFuncSetAttribute(step_fn<false>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute(step_fn<true>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(step_fn<false, true>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(step_fn<true, true>(fp64, team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

hipError_t launch_set_rows(float* dst, const float* src, const int* idx, int n, int n_actors, const int* table,
                           int field, int width, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const long long threads = (long long)n * kTeam;
  const int block = 256;
  const int grid = (int)((threads + block - 1) / block);
  hipLaunchKernelGGL(set_rows_kernel, dim3(grid), dim3(block), 0, stream, dst, src, idx, n, n_actors, table, field,
                     width);
  return hipGetLastError();
}

}  // namespace ags
