// FP64 CPU oracle for the batched articulated-physics step.
//
// TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and bench.py's CPU
// baseline.  Shares no code with the HIP library.
//
// Conventions (readings of what the paper leaves open; Section 2.3.2 fixes the tensor layouts):
//  * spatial vectors are [angular; linear] (Featherstone 2008, ch. 2);
//  * z is up, the ground plane is z = 0;
//  * a free root's link frame sits at its centre of mass; its generalized velocity is
//    (v_com world, omega world) and its generalized acceleration is the classical one;
//  * quaternions are xyzw (actor root state columns 3:7, Table 1 / Section 2.3.2 listing);
//  * one env-step = `substeps` substeps of h = dt / substeps with the controls held.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

namespace {

typedef std::array<double, 3> v3;
typedef std::array<double, 9> m3;   // row-major
typedef std::array<double, 6> v6;   // [angular; linear]
typedef std::array<double, 36> m6;  // row-major

// ---------------------------------------------------------------- 3-D algebra
v3 add(const v3& a, const v3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
v3 sub(const v3& a, const v3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
v3 scl(const v3& a, double s) { return {a[0] * s, a[1] * s, a[2] * s}; }
double dot(const v3& a, const v3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
v3 cross(const v3& a, const v3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const v3& a) { return std::sqrt(dot(a, a)); }
m3 eye3() { return {1, 0, 0, 0, 1, 0, 0, 0, 1}; }
m3 mmul(const m3& A, const m3& B) {
  m3 C{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) C[3 * i + j] += A[3 * i + k] * B[3 * k + j];
  return C;
}
m3 mT(const m3& A) {
  m3 B;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[3 * i + j] = A[3 * j + i];
  return B;
}
v3 mv(const m3& A, const v3& x) {
  return {A[0] * x[0] + A[1] * x[1] + A[2] * x[2], A[3] * x[0] + A[4] * x[1] + A[5] * x[2],
          A[6] * x[0] + A[7] * x[1] + A[8] * x[2]};
}
m3 skew(const v3& a) { return {0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0}; }
m3 madd(const m3& A, const m3& B) {
  m3 C;
  for (int i = 0; i < 9; ++i) C[i] = A[i] + B[i];
  return C;
}
m3 mscl(const m3& A, double s) {
  m3 C;
  for (int i = 0; i < 9; ++i) C[i] = A[i] * s;
  return C;
}
m3 outer(const v3& a, const v3& b) {
  m3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = a[i] * b[j];
  return C;
}

// Rodrigues: rotation by angle q about unit axis a (maps child coordinates to parent coordinates)
m3 axis_angle(const v3& a, double q) {
  double c = std::cos(q), s = std::sin(q);
  return madd(madd(mscl(eye3(), c), mscl(skew(a), s)), mscl(outer(a, a), 1.0 - c));
}

// quaternion (x, y, z, w) -> rotation matrix (body -> world); the quaternion is normalised first
m3 quat_to_mat(const double* qin) {
  double n = std::sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
  double x = qin[0] / n, y = qin[1] / n, z = qin[2] / n, w = qin[3] / n;
  return {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
          2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
          2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
}

// Hamilton product a (x) b, xyzw
std::array<double, 4> quat_mul(const std::array<double, 4>& a, const std::array<double, 4>& b) {
  v3 av = {a[0], a[1], a[2]}, bv = {b[0], b[1], b[2]};
  v3 v = add(add(scl(bv, a[3]), scl(av, b[3])), cross(av, bv));
  return {v[0], v[1], v[2], a[3] * b[3] - dot(av, bv)};
}

// ---------------------------------------------------------------- spatial algebra
v6 v6add(const v6& a, const v6& b) {
  v6 c;
  for (int i = 0; i < 6; ++i) c[i] = a[i] + b[i];
  return c;
}
v6 v6scl(const v6& a, double s) {
  v6 c;
  for (int i = 0; i < 6; ++i) c[i] = a[i] * s;
  return c;
}
double v6dot(const v6& a, const v6& b) {
  double s = 0;
  for (int i = 0; i < 6; ++i) s += a[i] * b[i];
  return s;
}
v6 m6v(const m6& A, const v6& x) {
  v6 y{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) y[i] += A[6 * i + j] * x[j];
  return y;
}
v6 m6Tv(const m6& A, const v6& x) {
  v6 y{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) y[j] += A[6 * i + j] * x[i];
  return y;
}
m6 m6mul(const m6& A, const m6& B) {
  m6 C{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      for (int k = 0; k < 6; ++k) C[6 * i + j] += A[6 * i + k] * B[6 * k + j];
  return C;
}
m6 m6T(const m6& A) {
  m6 B;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) B[6 * i + j] = A[6 * j + i];
  return B;
}
m6 m6add(const m6& A, const m6& B) {
  m6 C;
  for (int i = 0; i < 36; ++i) C[i] = A[i] + B[i];
  return C;
}
// X^T A X (congruence used to move an inertia from child to parent coordinates)
m6 congruence(const m6& X, const m6& A) { return m6mul(m6T(X), m6mul(A, X)); }

// Plucker motion transform from frame A to frame B: E rotates A coordinates into B coordinates and
// r is B's origin expressed in A (Featherstone eq. 2.24): X = [E 0; -E r^ E]
m6 plucker(const m3& E, const v3& r) {
  m3 Er = mscl(mmul(E, skew(r)), -1.0);
  m6 X{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      X[6 * i + j] = E[3 * i + j];
      X[6 * (i + 3) + (j + 3)] = E[3 * i + j];
      X[6 * (i + 3) + j] = Er[3 * i + j];
    }
  return X;
}
// motion cross product v x m
v6 crm(const v6& v, const v6& m) {
  v3 w = {v[0], v[1], v[2]}, vo = {v[3], v[4], v[5]};
  v3 mw = {m[0], m[1], m[2]}, mo = {m[3], m[4], m[5]};
  v3 a = cross(w, mw), b = add(cross(w, mo), cross(vo, mw));
  return {a[0], a[1], a[2], b[0], b[1], b[2]};
}
// force cross product v x* f
v6 crf(const v6& v, const v6& f) {
  v3 w = {v[0], v[1], v[2]}, vo = {v[3], v[4], v[5]};
  v3 n = {f[0], f[1], f[2]}, fo = {f[3], f[4], f[5]};
  v3 a = add(cross(w, n), cross(vo, fo)), b = cross(w, fo);
  return {a[0], a[1], a[2], b[0], b[1], b[2]};
}
// spatial inertia about a frame origin of a body with mass m, COM c and inertia Ic about the COM
// (Featherstone eq. 2.63): [Ic + m c^ c^T, m c^; m c^T, m 1]
m6 spatial_inertia(double m, const v3& c, const m3& Ic) {
  m3 C = skew(c);
  m3 A = madd(Ic, mscl(mmul(C, mT(C)), m));
  m6 I{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I[6 * i + j] = A[3 * i + j];
      I[6 * i + (j + 3)] = m * C[3 * i + j];
      I[6 * (i + 3) + j] = m * C[3 * j + i];
      I[6 * (i + 3) + (j + 3)] = (i == j) ? m : 0.0;
    }
  return I;
}

// ---------------------------------------------------------------- dense linear algebra
// Cholesky factorisation A = L L^T in place (lower triangle); false if not positive definite
bool cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
  }
  return true;
}
void chol_solve(const std::vector<double>& L, int n, std::vector<double>& x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
    x[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}
bool solve6(const m6& A, const v6& b, v6& x) {
  std::vector<double> L(A.begin(), A.end());
  if (!cholesky(L, 6)) return false;
  std::vector<double> y(b.begin(), b.end());
  chol_solve(L, 6, y);
  for (int i = 0; i < 6; ++i) x[i] = y[i];
  return true;
}

// ---------------------------------------------------------------- model
enum { J_FREE = 0, J_FIXED = 1, J_REV = 2, J_PRI = 3 };
enum { S_SPHERE = 0, S_CAPSULE = 1, S_BOX = 2 };

struct Shape {
  int kind, link;
  v3 p0, p1, half;
  double r, density;
};

struct Link {
  int parent, jtype;
  v3 anchor, axis;
  double lo, hi, kp, kd, armature, given_mass;
  std::vector<int> shapes;  // indices into Actor::shapes
  double m = 0.0;
  v3 com{};
  m3 Ic{};
  m6 I{};
  int col = -1;  // first generalized-velocity column (actor local); -1 for a fixed root
};

struct Actor {
  bool fixed = false;
  std::vector<Link> links;
  std::vector<Shape> shapes;
  int n_dof = 0, n_v = 0;
  int v_off = 0, dof_off = 0, body_off = 0;
};

struct Pair {
  int aa, al, as, ba, bl, bs;  // as/bs are actor-local shape indices
};

// fixed tendon (appendix on tendons): a tree of tendon joints, each following one DOF with a coefficient;
// the length at a tendon joint is its parent's length plus coefficient x joint position
struct Tendon {
  std::vector<int> dof, parent;  // per tendon joint: env DOF index, parent tendon joint (-1 root)
  std::vector<double> coef;
  double k, d, rest, lo, hi, klim;
};

struct Env {
  std::vector<Actor> actors;
  std::vector<Pair> pairs;
  std::vector<Tendon> tendons;
  int n_dof = 0, n_v = 0, n_bodies = 0, n_slots = 0, max_rows = 0;
};

// mass properties of one shape about its own centroid, in the link frame (closed forms)
void shape_mass(const Shape& s, double rho, double& m, v3& c, m3& Ic) {
  const double pi = 3.14159265358979323846;
  if (s.kind == S_SPHERE) {
    m = rho * 4.0 / 3.0 * pi * s.r * s.r * s.r;
    c = s.p0;
    Ic = mscl(eye3(), 0.4 * m * s.r * s.r);
  } else if (s.kind == S_CAPSULE) {
    // cylinder of length L plus two hemispherical caps; a hemisphere's COM lies 3r/8 from its base and
    // its inertia about a diameter through that COM is (83/320) m_hemi r^2
    v3 d = sub(s.p1, s.p0);
    double L = norm(d), r = s.r;
    double mc = rho * pi * r * r * L;
    double mh = rho * 4.0 / 3.0 * pi * r * r * r;  // both caps together
    m = mc + mh;
    c = scl(add(s.p0, s.p1), 0.5);
    double Iax = mc * r * r / 2.0 + mh * 0.4 * r * r;
    double off = L / 2.0 + 3.0 * r / 8.0;
    double Iperp = mc * (r * r / 4.0 + L * L / 12.0) + mh * (83.0 / 320.0 * r * r + off * off);
    v3 u = L > 0 ? scl(d, 1.0 / L) : v3{0, 0, 1};
    Ic = madd(mscl(eye3(), Iperp), mscl(outer(u, u), Iax - Iperp));
  } else {
    double a = s.half[0], b = s.half[1], cc = s.half[2];
    m = rho * 8.0 * a * b * cc;
    c = s.p0;
    Ic = {m / 3.0 * (b * b + cc * cc), 0, 0, 0, m / 3.0 * (a * a + cc * cc), 0, 0, 0, m / 3.0 * (a * a + b * b)};
  }
}

bool compile_actor(Actor& A, std::string& err) {
  int col = 0;
  if (A.links.empty()) { err = "actor without links"; return false; }
  A.fixed = A.links[0].jtype == J_FIXED;
  if (!A.fixed) { A.links[0].col = 0; col = 6; }
  for (size_t i = 0; i < A.links.size(); ++i) {
    Link& L = A.links[i];
    if (i == 0 && (L.parent != -1 || (L.jtype != J_FREE && L.jtype != J_FIXED))) { err = "bad root"; return false; }
    if (i > 0 && (L.parent < 0 || L.parent >= (int)i || (L.jtype != J_REV && L.jtype != J_PRI))) {
      err = "links must be topologically ordered 1-DOF joints"; return false;
    }
    if (i > 0) { L.col = col++; }
    // mass properties
    double msum = 0; v3 csum{}; std::vector<double> ms; std::vector<v3> cs; std::vector<m3> Is;
    for (int si : L.shapes) {
      double m; v3 c; m3 Ic;
      shape_mass(A.shapes[si], A.shapes[si].density, m, c, Ic);
      ms.push_back(m); cs.push_back(c); Is.push_back(Ic);
      msum += m; csum = add(csum, scl(c, m));
    }
    L.m = msum;
    L.com = msum > 0 ? scl(csum, 1.0 / msum) : v3{0, 0, 0};
    L.Ic = m3{};
    for (size_t k = 0; k < ms.size(); ++k) {
      v3 d = sub(cs[k], L.com);
      // parallel-axis theorem: I += m (|d|^2 1 - d d^T)
      L.Ic = madd(L.Ic, madd(Is[k], mscl(madd(mscl(eye3(), dot(d, d)), mscl(outer(d, d), -1.0)), ms[k])));
    }
    if (L.given_mass > 0) {
      if (msum <= 0) { err = "given mass on a link without shapes"; return false; }
      double s = L.given_mass / msum;
      L.m = L.given_mass;
      L.Ic = mscl(L.Ic, s);
    }
    L.I = spatial_inertia(L.m, L.com, L.Ic);
  }
  if (!A.fixed && norm(A.links[0].com) > 1e-9) { err = "free root link frame must sit at its centre of mass"; return false; }
  if (!A.fixed && A.links[0].m <= 0) { err = "free root without mass"; return false; }
  A.n_dof = (int)A.links.size() - 1;
  A.n_v = col;
  return true;
}

int slots_of_pair(const Env& E, const Pair& p) {
  const Shape& s = E.actors[p.aa].shapes[p.as];
  if (p.ba < 0) return s.kind == S_SPHERE ? 1 : (s.kind == S_CAPSULE ? 2 : 8);
  return s.kind == S_SPHERE ? 1 : 3;  // sphere-box 1, capsule-box 3 (two caps + segment midpoint)
}

// ---------------------------------------------------------------- kinematics
struct Kin {
  std::vector<m3> R;   // link -> world rotation
  std::vector<v3> p;   // link origin, world
  std::vector<m6> X;   // parent -> link Plucker transform (root: world -> link)
  std::vector<v6> S;   // joint motion subspace in link coordinates (non-root)
};

void kinematics(const Actor& A, const double* root, const double* q, Kin& K) {
  size_t n = A.links.size();
  K.R.resize(n); K.p.resize(n); K.X.resize(n); K.S.resize(n);
  K.R[0] = quat_to_mat(root + 3);
  K.p[0] = {root[0], root[1], root[2]};
  K.X[0] = plucker(mT(K.R[0]), K.p[0]);
  for (size_t i = 1; i < n; ++i) {
    const Link& L = A.links[i];
    double qi = q[i - 1];
    m3 Rrel = L.jtype == J_REV ? axis_angle(L.axis, qi) : eye3();
    v3 t = L.jtype == J_PRI ? add(L.anchor, scl(L.axis, qi)) : L.anchor;
    K.X[i] = plucker(mT(Rrel), t);
    K.R[i] = mmul(K.R[L.parent], Rrel);
    K.p[i] = add(K.p[L.parent], mv(K.R[L.parent], t));
    K.S[i] = L.jtype == J_REV ? v6{L.axis[0], L.axis[1], L.axis[2], 0, 0, 0} : v6{0, 0, 0, L.axis[0], L.axis[1], L.axis[2]};
  }
}

// gravity as an external spatial force on each link, in link coordinates
v6 gravity_force(const Link& L, const m3& R, const v3& g) {
  v3 F = mv(mT(R), scl(g, L.m));
  v3 n = cross(L.com, F);
  return {n[0], n[1], n[2], F[0], F[1], F[2]};
}

// free-root spatial velocity in root coordinates from (v_com, omega) in world
v6 root_velocity(const m3& R, const double* qd) {
  v3 vc = {qd[0], qd[1], qd[2]}, w = {qd[3], qd[4], qd[5]};
  v3 wb = mv(mT(R), w), vb = mv(mT(R), vc);
  return {wb[0], wb[1], wb[2], vb[0], vb[1], vb[2]};
}

// RNEA (Featherstone Table 5.1) with the floating base as a 6-DOF joint: returns generalized forces
void rnea(const Actor& A, const Kin& K, const double* qd, const double* qdd, const v3& g, double* tau) {
  size_t n = A.links.size();
  std::vector<v6> v(n), a(n), f(n);
  for (size_t i = 0; i < n; ++i) {
    const Link& L = A.links[i];
    if (i == 0) {
      if (A.fixed) { v[0] = v6{}; a[0] = v6{}; }
      else {
        v[0] = root_velocity(K.R[0], qd);
        v3 vc = {qd[0], qd[1], qd[2]}, w = {qd[3], qd[4], qd[5]};
        v3 vcd = {qdd[0], qdd[1], qdd[2]}, wd = {qdd[3], qdd[4], qdd[5]};
        // spatial acceleration at the COM: [R^T wd; R^T (vcd - w x vc)]
        v3 ab = mv(mT(K.R[0]), wd), lb = mv(mT(K.R[0]), sub(vcd, cross(w, vc)));
        a[0] = {ab[0], ab[1], ab[2], lb[0], lb[1], lb[2]};
      }
    } else {
      double qdi = qd[L.col], qddi = qdd[L.col];
      v[i] = v6add(m6v(K.X[i], v[L.parent]), v6scl(K.S[i], qdi));
      a[i] = v6add(v6add(m6v(K.X[i], a[L.parent]), v6scl(K.S[i], qddi)), crm(v[i], v6scl(K.S[i], qdi)));
    }
    v6 fg = gravity_force(L, K.R[i], g);
    f[i] = v6add(v6add(m6v(L.I, a[i]), crf(v[i], m6v(L.I, v[i]))), v6scl(fg, -1.0));
  }
  for (size_t i = n - 1; i >= 1; --i) {
    const Link& L = A.links[i];
    tau[L.col] = v6dot(K.S[i], f[i]);
    f[L.parent] = v6add(f[L.parent], m6Tv(K.X[i], f[i]));
  }
  if (!A.fixed) {
    v3 n0 = {f[0][0], f[0][1], f[0][2]}, f0 = {f[0][3], f[0][4], f[0][5]};
    v3 F = mv(K.R[0], f0), N = mv(K.R[0], n0);
    for (int k = 0; k < 3; ++k) { tau[k] = F[k]; tau[3 + k] = N[k]; }
  }
}

// columns of the free-root joint: maps (v_com, omega) world to the root spatial velocity
m6 root_subspace(const m3& R) {
  m3 Rt = mT(R);
  m6 S{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S[6 * i + (j + 3)] = Rt[3 * i + j];
      S[6 * (i + 3) + j] = Rt[3 * i + j];
    }
  return S;
}

// CRBA (Featherstone Table 6.2): joint-space inertia of one actor into M (ld = leading dimension)
void crba(const Actor& A, const Kin& K, double* M, int ld) {
  size_t n = A.links.size();
  std::vector<m6> Ic(n);
  for (size_t i = 0; i < n; ++i) Ic[i] = A.links[i].I;
  for (size_t i = n - 1; i >= 1; --i) Ic[A.links[i].parent] = m6add(Ic[A.links[i].parent], congruence(K.X[i], Ic[i]));
  auto subspace_cols = [&](size_t i, std::vector<v6>& cols) {
    cols.clear();
    if (i == 0) {
      m6 S0 = root_subspace(K.R[0]);
      for (int c = 0; c < 6; ++c) cols.push_back({S0[c], S0[6 + c], S0[12 + c], S0[18 + c], S0[24 + c], S0[30 + c]});
    } else {
      cols.push_back(K.S[i]);
    }
  };
  std::vector<v6> Si, Sj;
  for (size_t i = 0; i < n; ++i) {
    if (i == 0 && A.fixed) continue;
    subspace_cols(i, Si);
    std::vector<v6> F(Si.size());
    for (size_t c = 0; c < Si.size(); ++c) F[c] = m6v(Ic[i], Si[c]);
    int ci = A.links[i].col;
    for (size_t a = 0; a < Si.size(); ++a)
      for (size_t b = 0; b < Si.size(); ++b) M[(ci + a) * ld + ci + b] = v6dot(Si[a], F[b]);
    size_t j = i;
    while (j > 0) {
      for (auto& Fc : F) Fc = m6Tv(K.X[j], Fc);
      j = A.links[j].parent;
      if (j == 0 && A.fixed) break;
      subspace_cols(j, Sj);
      int cj = A.links[j].col;
      for (size_t a = 0; a < Si.size(); ++a)
        for (size_t b = 0; b < Sj.size(); ++b) {
          double h = v6dot(F[a], Sj[b]);
          M[(ci + a) * ld + cj + b] = h;
          M[(cj + b) * ld + ci + a] = h;
        }
    }
  }
}

// ABA (Featherstone Table 7.1) with the floating base as a 6-DOF joint.  Kept as a self-check of
// CRBA + RNEA + Cholesky; armature[col] is added to the joint's D.
void aba(const Actor& A, const Kin& K, const double* qd, const double* tau, const double* armature, const v3& g,
         double* qdd) {
  size_t n = A.links.size();
  std::vector<v6> v(n), c(n), pA(n), U(n), a(n);
  std::vector<m6> IA(n);
  std::vector<double> D(n), u(n);
  for (size_t i = 0; i < n; ++i) {
    const Link& L = A.links[i];
    if (i == 0) {
      if (A.fixed) { v[0] = v6{}; c[0] = v6{}; }
      else {
        v[0] = root_velocity(K.R[0], qd);
        v3 vc = {qd[0], qd[1], qd[2]}, w = {qd[3], qd[4], qd[5]};
        v3 lb = mv(mT(K.R[0]), scl(cross(w, vc), -1.0));
        c[0] = {0, 0, 0, lb[0], lb[1], lb[2]};
      }
    } else {
      v6 vJ = v6scl(K.S[i], qd[L.col]);
      v[i] = v6add(m6v(K.X[i], v[L.parent]), vJ);
      c[i] = crm(v[i], vJ);
    }
    IA[i] = L.I;
    pA[i] = v6add(crf(v[i], m6v(L.I, v[i])), v6scl(gravity_force(L, K.R[i], g), -1.0));
  }
  for (size_t i = n - 1; i >= 1; --i) {
    const Link& L = A.links[i];
    U[i] = m6v(IA[i], K.S[i]);
    D[i] = v6dot(K.S[i], U[i]) + armature[L.col];
    u[i] = tau[L.col] - v6dot(K.S[i], pA[i]);
    m6 Ia = IA[i];
    for (int r = 0; r < 6; ++r)
      for (int s = 0; s < 6; ++s) Ia[6 * r + s] -= U[i][r] * U[i][s] / D[i];
    v6 pa = v6add(v6add(pA[i], m6v(Ia, c[i])), v6scl(U[i], u[i] / D[i]));
    IA[L.parent] = m6add(IA[L.parent], congruence(K.X[i], Ia));
    pA[L.parent] = v6add(pA[L.parent], m6Tv(K.X[i], pa));
  }
  if (A.fixed) {
    a[0] = v6{};
  } else {
    // the root's total spatial acceleration solves IA0 a0 + pA0 = 0
    v6 rhs = v6scl(pA[0], -1.0);
    solve6(IA[0], rhs, a[0]);
    v6 s = m6Tv(root_subspace(K.R[0]), v6add(a[0], v6scl(c[0], -1.0)));  // S0^-1 = S0^T
    for (int k = 0; k < 6; ++k) qdd[k] = s[k];
  }
  for (size_t i = 1; i < n; ++i) {
    const Link& L = A.links[i];
    v6 ap = v6add(m6v(K.X[i], a[L.parent]), c[i]);
    qdd[L.col] = (u[i] - v6dot(U[i], ap)) / D[i];
    a[i] = v6add(ap, v6scl(K.S[i], qdd[L.col]));
  }
}

// linear velocity (world) of the body point at world position x, per generalized velocity column:
// fills Jp (3 x n_v_env, row-major with leading dimension ld) for body (actor, link), sign s
void point_jacobian(const Env& E, int actor, int link, const std::vector<Kin>& K, const v3& x, double s,
                    double* Jp, int ld) {
  const Actor& A = E.actors[actor];
  const Kin& k = K[actor];
  int off = A.v_off;
  int i = link;
  while (true) {
    const Link& L = A.links[i];
    if (i == 0) {
      if (!A.fixed) {
        // u = v_c + omega x (x - c): columns I (for v_c) and e_m x (x - c) (for omega_m)
        v3 r = sub(x, k.p[0]);
        for (int m = 0; m < 3; ++m) {
          Jp[m * ld + off + m] += s;
          v3 e{0, 0, 0}; e[m] = 1;
          v3 col = cross(e, r);
          for (int row = 0; row < 3; ++row) Jp[row * ld + off + 3 + m] += s * col[row];
        }
      }
      break;
    }
    v3 a = mv(k.R[i], L.axis);  // world joint axis
    v3 col = L.jtype == J_REV ? cross(a, sub(x, k.p[i])) : a;
    for (int row = 0; row < 3; ++row) Jp[row * ld + off + L.col] += s * col[row];
    i = L.parent;
  }
}

// ---------------------------------------------------------------- narrow phase
struct Slot {
  int pair, slot;
  int a_actor, a_link, b_actor, b_link;  // b_actor -1: ground
  double phi;
  v3 n, x;   // normal (from b towards a) and contact point on body a's surface
  int near;  // geometric ambiguity flags
};

v3 world_point(const Kin& k, int link, const v3& local) { return add(k.p[link], mv(k.R[link], local)); }

// sphere (centre x, radius r) against a box (pose Rb, cb, half extents h): closest-point rule, or the face
// of least penetration when the centre is inside (ties: lowest axis, then the + side)
void sphere_box(const v3& x, double r, const m3& Rb, const v3& cb, const v3& h, double& phi, v3& n, int& near) {
  near = 0;
  v3 xl = mv(mT(Rb), sub(x, cb));
  v3 ql;
  bool inside = true;
  for (int k = 0; k < 3; ++k) {
    ql[k] = std::min(std::max(xl[k], -h[k]), h[k]);
    if (xl[k] != ql[k]) inside = false;
  }
  v3 dl = sub(xl, ql);
  double d = norm(dl);
  if (!inside && d > 1e-12) {
    phi = d - r;
    n = mv(Rb, scl(dl, 1.0 / d));
    if (d < 1e-5) near |= ORC_NEAR_GEOM;
  } else {
    int kbest = 0;
    double pen[3];
    for (int k = 0; k < 3; ++k) pen[k] = h[k] - std::fabs(xl[k]);
    for (int k = 1; k < 3; ++k)
      if (pen[k] < pen[kbest]) kbest = k;
    for (int k = 0; k < 3; ++k)
      if (k != kbest && std::fabs(pen[k] - pen[kbest]) < 1e-5) near |= ORC_NEAR_GEOM;
    if (pen[kbest] < 1e-5) near |= ORC_NEAR_GEOM;
    v3 nl{0, 0, 0};
    nl[kbest] = xl[kbest] >= 0 ? 1.0 : -1.0;
    if (std::fabs(xl[kbest]) < 1e-5) near |= ORC_NEAR_GEOM;
    phi = -pen[kbest] - r;
    n = mv(Rb, nl);
  }
}

void narrow_phase(const Env& E, const std::vector<Kin>& K, std::vector<Slot>& out) {
  out.clear();
  for (size_t pi = 0; pi < E.pairs.size(); ++pi) {
    const Pair& P = E.pairs[pi];
    const Actor& A = E.actors[P.aa];
    const Shape& s = A.shapes[P.as];
    const Kin& ka = K[P.aa];
    std::vector<std::pair<v3, double>> spheres;  // body-a spheres (centre world, radius)
    if (s.kind == S_SPHERE) spheres.push_back({world_point(ka, s.link, s.p0), s.r});
    if (s.kind == S_CAPSULE) {
      spheres.push_back({world_point(ka, s.link, s.p0), s.r});
      spheres.push_back({world_point(ka, s.link, s.p1), s.r});
      if (P.ba >= 0) spheres.push_back({world_point(ka, s.link, scl(add(s.p0, s.p1), 0.5)), s.r});
    }
    if (P.ba < 0) {
      v3 up = {0, 0, 1};
      if (s.kind == S_BOX) {
        for (int c = 0; c < 8; ++c) {
          v3 corner = {s.p0[0] + ((c & 1) ? s.half[0] : -s.half[0]), s.p0[1] + ((c & 2) ? s.half[1] : -s.half[1]),
                       s.p0[2] + ((c & 4) ? s.half[2] : -s.half[2])};
          v3 x = world_point(ka, s.link, corner);
          out.push_back({(int)pi, c, P.aa, s.link, -1, -1, x[2], up, x, 0});
        }
      } else {
        for (size_t c = 0; c < spheres.size(); ++c) {
          v3 x = spheres[c].first;
          double r = spheres[c].second;
          out.push_back({(int)pi, (int)c, P.aa, s.link, -1, -1, x[2] - r, up, sub(x, scl(up, r)), 0});
        }
      }
    } else {
      const Actor& B = E.actors[P.ba];
      const Shape& sb = B.shapes[P.bs];
      const Kin& kb = K[P.ba];
      m3 Rb = kb.R[sb.link];
      v3 cb = world_point(kb, sb.link, sb.p0);
      for (size_t c = 0; c < spheres.size(); ++c) {
        double phi; v3 n; int near;
        sphere_box(spheres[c].first, spheres[c].second, Rb, cb, sb.half, phi, n, near);
        v3 x = sub(spheres[c].first, scl(n, spheres[c].second));
        out.push_back({(int)pi, (int)c, P.aa, s.link, P.ba, sb.link, phi, n, x, near});
      }
    }
  }
}

// tangent basis: t1 = normalised projection of the world axis least aligned with n (lowest index on ties)
void tangents(const v3& n, v3& t1, v3& t2, int& near) {
  int k = 0;
  double best = std::fabs(n[0]);
  for (int i = 1; i < 3; ++i)
    if (std::fabs(n[i]) < best) { best = std::fabs(n[i]); k = i; }
  for (int i = 0; i < 3; ++i)
    // exact ties (e.g. the plane normal +z) break identically in any precision; near ties do not
    if (i != k && std::fabs(n[i]) != best && std::fabs(std::fabs(n[i]) - best) < 1e-6) near |= ORC_NEAR_TANGENT;
  v3 e{0, 0, 0}; e[k] = 1;
  v3 t = sub(e, scl(n, dot(n, e)));
  t1 = scl(t, 1.0 / norm(t));
  t2 = cross(n, t1);
}

// ---------------------------------------------------------------- one env, one step
struct Params {
  double dt, h, beta, mu, mc, ml_rev, ml_pri, guard_c, guard_l;
  int substeps, iters;
  int tgs;  // 1: temporal Gauss-Seidel variant
  v3 g;
};

struct Row {
  int key, kind;      // kind 1/2 limit, 3 normal, 4/5 tangents
  int branch = 0;     // bias branch: 1 when the gap is negative (Baumgarte), 0 when speculative
  int normal_row;     // tangent rows: index of their normal row
  int slot;           // contact rows: index into the slot list
  std::vector<double> J, W;
  double bias, A;
  double pos = 0.0;   // limit and contact-normal rows: the position error (gap or phi) the bias comes from
};

struct StepOut {
  double* qdd_free; int r_cap; int* row_count; int* row_key; double* row_lambda;
  double* contact_force; double* contact_scale; double* dof_force; int* near; unsigned long long* mode;
};

// FNV-1a over the discrete decisions of a step
struct ModeHash {
  unsigned long long h = 1469598103934665603ull;
  void mix(long long v) {
    h ^= (unsigned long long)v;
    h *= 1099511628211ull;
  }
};

// unpack env state into per-actor root arrays and the env generalized vectors
void split_state(const Env& E, const double* root, const double* dof, std::vector<double>& qj,
                 std::vector<double>& qd) {
  qj.assign(E.n_dof, 0.0);
  qd.assign(E.n_v, 0.0);
  for (size_t ai = 0; ai < E.actors.size(); ++ai) {
    const Actor& A = E.actors[ai];
    if (!A.fixed)
      for (int k = 0; k < 6; ++k) qd[A.v_off + k] = root[13 * ai + 7 + k];
    for (int j = 0; j < A.n_dof; ++j) {
      qj[A.dof_off + j] = dof[2 * (A.dof_off + j)];
      qd[A.v_off + A.links[j + 1].col] = dof[2 * (A.dof_off + j) + 1];
    }
  }
}

void step_env(const Env& E, const Params& P, const double* root_in, const double* dof_in, const double* act,
              const double* pos_tgt, const double* vel_tgt, double* root_out, double* dof_out, const StepOut& O) {
  const int nv = E.n_v, nd = E.n_dof, na = (int)E.actors.size();
  std::vector<double> root(root_in, root_in + 13 * na);
  std::vector<double> qj, qd;
  split_state(E, root.data(), dof_in, qj, qd);
  // env DOF index -> generalized column, joint type, limits, drive
  std::vector<int> dcol(nd), dtype(nd);
  std::vector<const Link*> dlink(nd);
  for (const Actor& A : E.actors)
    for (int j = 0; j < A.n_dof; ++j) {
      dcol[A.dof_off + j] = A.v_off + A.links[j + 1].col;
      dtype[A.dof_off + j] = A.links[j + 1].jtype;
      dlink[A.dof_off + j] = &A.links[j + 1];
    }
  std::vector<double> cforce(3 * E.n_bodies, 0.0), cscale(2 * E.n_bodies, 0.0), dforce(nd, 0.0);
  const double h = P.h;
  ModeHash mode;

  for (int sub = 0; sub < P.substeps; ++sub) {
    // kinematics of every actor at the current state
    std::vector<Kin> K(na);
    for (int ai = 0; ai < na; ++ai) kinematics(E.actors[ai], &root[13 * ai], &qj[E.actors[ai].dof_off], K[ai]);
    // generalized forces: actuation plus the explicit part of the implicit PD drive; armature
    // a~ = armature + h kd + h^2 kp enters M~ (the drive evaluated at the end-of-substep state)
    std::vector<double> tau(nv, 0.0), arm(nv, 0.0);
    for (int j = 0; j < nd; ++j) {
      const Link* L = dlink[j];
      int c = dcol[j];
      tau[c] = act[j] + L->kp * (pos_tgt[j] - qj[j] - h * qd[c]) + L->kd * (vel_tgt[j] - qd[c]);
      arm[c] = L->armature + h * L->kd + h * h * L->kp;
    }
    // fixed tendons: at each tendon joint a spring-damper on the length l (stiffness k about the rest length,
    // damping d on dl/dt) plus a limit spring klim beyond [lo, hi]; the force f acts on every DOF of the path
    // from the tendon's root to that joint as the generalized force -f dl/dq = -f coef
    for (const Tendon& T : E.tendons) {
      const int n = (int)T.dof.size();
      std::vector<double> len(n), rate(n);
      for (int j = 0; j < n; ++j) {
        const int c = dcol[T.dof[j]];
        len[j] = (T.parent[j] >= 0 ? len[T.parent[j]] : 0.0) + T.coef[j] * qj[T.dof[j]];
        rate[j] = (T.parent[j] >= 0 ? rate[T.parent[j]] : 0.0) + T.coef[j] * qd[c];
      }
      for (int j = 0; j < n; ++j) {
        double f = T.k * (len[j] - T.rest) + T.d * rate[j];
        if (len[j] > T.hi) f += T.klim * (len[j] - T.hi);
        if (len[j] < T.lo) f += T.klim * (len[j] - T.lo);
        for (int p = j; p >= 0; p = T.parent[p]) tau[dcol[T.dof[p]]] -= f * T.coef[p];
      }
    }
    // M~ = blockdiag(M_actor) + diag(a~);  C from RNEA with qdd = 0
    std::vector<double> M(nv * nv, 0.0), C(nv, 0.0), zero(nv, 0.0);
    for (int ai = 0; ai < na; ++ai) {
      const Actor& A = E.actors[ai];
      crba(A, K[ai], &M[A.v_off * nv + A.v_off], nv);
      rnea(A, K[ai], &qd[A.v_off], &zero[A.v_off], P.g, &C[A.v_off]);
    }
    for (int c = 0; c < nv; ++c) M[c * nv + c] += arm[c];
    std::vector<double> L = M;
    cholesky(L, nv);
    std::vector<double> qdd(nv);
    for (int c = 0; c < nv; ++c) qdd[c] = tau[c] - C[c];
    chol_solve(L, nv, qdd);
    if (O.qdd_free)
      for (int c = 0; c < nv; ++c) O.qdd_free[sub * nv + c] = qdd[c];
    std::vector<double> vstar(nv);
    for (int c = 0; c < nv; ++c) vstar[c] = qd[c] + h * qdd[c];

    int near = 0;
    // ---- rows: joint limits first (by DOF, lower before upper), then contacts (pair, slot; n, t1, t2)
    std::vector<Row> rows;
    for (int j = 0; j < nd; ++j) {
      const Link* Lk = dlink[j];
      double ml = dtype[j] == J_PRI ? P.ml_pri : P.ml_rev;
      int c = dcol[j];
      for (int side = 0; side < 2; ++side) {
        double bound = side == 0 ? Lk->lo : Lk->hi;
        if (!std::isfinite(bound)) continue;
        double gap = side == 0 ? qj[j] - bound : bound - qj[j];
        double rate = side == 0 ? vstar[c] : -vstar[c];
        double act_gap = std::min(gap, gap + h * rate);
        if (std::fabs(act_gap - ml) < P.guard_l) near |= ORC_NEAR_LIMIT;
        if (!(act_gap < ml)) continue;
        Row r;
        r.kind = side == 0 ? 1 : 2;
        r.key = (r.kind << 24) | (j << 8);
        r.normal_row = -1; r.slot = -1;
        r.J.assign(nv, 0.0);
        r.J[c] = side == 0 ? 1.0 : -1.0;
        r.bias = gap >= 0 ? gap / h : P.beta * gap / h;
        r.branch = gap >= 0 ? 0 : 1;
        r.pos = gap;
        rows.push_back(r);
      }
    }
    std::vector<Slot> slots;
    narrow_phase(E, K, slots);
    std::vector<double> Jp(3 * nv);
    for (size_t si = 0; si < slots.size(); ++si) {
      const Slot& s = slots[si];
      std::fill(Jp.begin(), Jp.end(), 0.0);
      point_jacobian(E, s.a_actor, s.a_link, K, s.x, 1.0, Jp.data(), nv);
      if (s.b_actor >= 0) point_jacobian(E, s.b_actor, s.b_link, K, s.x, -1.0, Jp.data(), nv);
      double vn = 0;
      for (int c = 0; c < nv; ++c) vn += (s.n[0] * Jp[c] + s.n[1] * Jp[nv + c] + s.n[2] * Jp[2 * nv + c]) * vstar[c];
      double act_gap = s.phi + h * std::min(0.0, vn);
      if (std::fabs(act_gap - P.mc) < P.guard_c) near |= ORC_NEAR_CONTACT;
      if (!(act_gap < P.mc)) continue;
      near |= s.near;
      v3 t1, t2;
      tangents(s.n, t1, t2, near);
      v3 dirs[3] = {s.n, t1, t2};
      int nrow = (int)rows.size();
      for (int k = 0; k < 3; ++k) {
        Row r;
        r.kind = 3 + k;
        r.key = (r.kind << 24) | (s.pair << 8) | s.slot;
        r.normal_row = k == 0 ? -1 : nrow;
        r.slot = (int)si;
        r.J.assign(nv, 0.0);
        for (int c = 0; c < nv; ++c)
          r.J[c] = dirs[k][0] * Jp[c] + dirs[k][1] * Jp[nv + c] + dirs[k][2] * Jp[2 * nv + c];
        r.bias = k == 0 ? (s.phi >= 0 ? s.phi / h : P.beta * s.phi / h) : 0.0;
        r.branch = k == 0 && s.phi < 0 ? 1 : 0;
        r.pos = k == 0 ? s.phi : 0.0;
        rows.push_back(r);
      }
    }
    // ---- coupling: W_r = M~^-1 J_r^T, A_rr = J_r W_r; rows with A_rr below 1e-6 are dropped
    std::vector<Row> kept;
    std::vector<int> remap(rows.size(), -1);
    for (size_t ri = 0; ri < rows.size(); ++ri) {
      Row& r = rows[ri];
      r.W = r.J;
      chol_solve(L, nv, r.W);
      r.A = 0;
      for (int c = 0; c < nv; ++c) r.A += r.J[c] * r.W[c];
      if (std::fabs(r.A - 1e-6) < 1e-7) near |= ORC_NEAR_SKIP;
      if (!(r.A >= 1e-6)) continue;
      if (r.kind >= 4 && remap[r.normal_row] < 0) continue;
      remap[ri] = (int)kept.size();
      if (r.kind >= 4) r.normal_row = remap[r.normal_row];
      kept.push_back(r);
    }
    for (const Row& r : kept) {
      mode.mix(r.key);
      mode.mix(r.branch);
    }
    mode.mix(-1);
    // ---- projected Gauss-Seidel: fixed sweeps from lambda = 0, v = v*.  Temporal variant (Section 3):
    // the velocity at the end of each sweep, times h / iters, is accumulated into a displacement; a limit
    // or contact-normal row's bias is that of its position error plus the displacement along its row
    // (the same two branches as above), recomputed before every sweep.
    std::vector<double> lam(kept.size(), 0.0), v = vstar, disp(nv, 0.0);
    for (int it = 0; it < P.iters; ++it) {
      if (P.tgs) {
        for (Row& r : kept) {
          if (r.kind >= 4) continue;
          double C = r.pos;
          for (int c = 0; c < nv; ++c) C += r.J[c] * disp[c];
          r.bias = C >= 0 ? C / h : P.beta * C / h;
          mode.mix(C >= 0 ? 0 : 1);  // the bias is continuous in C; only its slope switches
        }
      }
      for (size_t ri = 0; ri < kept.size(); ++ri) {
        const Row& r = kept[ri];
        double res = r.bias;
        for (int c = 0; c < nv; ++c) res += r.J[c] * v[c];
        double x = lam[ri] - res / r.A;
        double lo = 0.0, hi = INFINITY;
        if (r.kind >= 4) { hi = P.mu * lam[r.normal_row]; lo = -hi; }
        double nl = std::min(std::max(x, lo), hi);
        mode.mix(x > hi ? 2 : (x < lo ? 1 : 0));
        if (std::fabs(x - lo) < 1e-6 * (1.0 + std::fabs(lo)) || std::fabs(x - hi) < 1e-6 * (1.0 + std::fabs(hi)))
          near |= ORC_NEAR_CLAMP;
        double dl = nl - lam[ri];
        for (int c = 0; c < nv; ++c) v[c] += r.W[c] * dl;
        lam[ri] = nl;
      }
      if (P.tgs)
        for (int c = 0; c < nv; ++c) disp[c] += h / P.iters * v[c];
    }
    if (O.row_count) O.row_count[sub] = (int)kept.size();
    for (size_t ri = 0; ri < kept.size() && (int)ri < O.r_cap; ++ri) {
      if (O.row_key) O.row_key[sub * O.r_cap + ri] = kept[ri].key;
      if (O.row_lambda) O.row_lambda[sub * O.r_cap + ri] = lam[ri];
    }
    if (O.near) O.near[sub] = near;
    // contact impulses -> forces on bodies (partner gets the opposite), summed over substeps / dt
    for (size_t ri = 0; ri < kept.size(); ++ri) {
      const Row& r = kept[ri];
      if (r.kind < 3) continue;
      const Slot& s = slots[r.slot];
      v3 d;
      if (r.kind == 3) d = s.n;
      else { v3 t1, t2; int dummy = 0; tangents(s.n, t1, t2, dummy); d = r.kind == 4 ? t1 : t2; }
      v3 F = scl(d, lam[ri] / P.dt);
      int ba = E.actors[s.a_actor].body_off + s.a_link;
      for (int k = 0; k < 3; ++k) cforce[3 * ba + k] += F[k];
      cscale[2 * ba] += 1.0;
      cscale[2 * ba + 1] += std::fabs(lam[ri]) / P.dt;
      if (s.b_actor >= 0) {
        int bb = E.actors[s.b_actor].body_off + s.b_link;
        for (int k = 0; k < 3; ++k) cforce[3 * bb + k] -= F[k];
        cscale[2 * bb] += 1.0;
        cscale[2 * bb + 1] += std::fabs(lam[ri]) / P.dt;
      }
    }
    // ---- semi-implicit integration: qd+ = v; q+ = q + h qd+; root quat+ = normalize(Exp(h w+) (x) quat)
    for (int j = 0; j < nd; ++j) {
      const Link* Lk = dlink[j];
      int c = dcol[j];
      dforce[j] += act[j] + Lk->kp * (pos_tgt[j] - qj[j] - h * v[c]) + Lk->kd * (vel_tgt[j] - v[c]);
      qj[j] += h * v[c];
    }
    for (int ai = 0; ai < na; ++ai) {
      const Actor& A = E.actors[ai];
      double* rs = &root[13 * ai];
      if (A.fixed) continue;
      const double* vr = &v[A.v_off];
      for (int k = 0; k < 3; ++k) rs[k] += h * vr[k];
      v3 th = {h * vr[3], h * vr[4], h * vr[5]};
      double ang = norm(th);
      std::array<double, 4> dq;
      if (ang < 1e-8) {
        dq = {th[0] / 2, th[1] / 2, th[2] / 2, 1.0};
      } else {
        double s = std::sin(ang / 2) / ang;
        dq = {th[0] * s, th[1] * s, th[2] * s, std::cos(ang / 2)};
      }
      std::array<double, 4> q0 = {rs[3], rs[4], rs[5], rs[6]};
      std::array<double, 4> q1 = quat_mul(dq, q0);
      double qn = std::sqrt(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2] + q1[3] * q1[3]);
      for (int k = 0; k < 4; ++k) rs[3 + k] = q1[k] / qn;
      for (int k = 0; k < 6; ++k) rs[7 + k] = vr[k];
    }
    for (int c = 0; c < nv; ++c) qd[c] = v[c];
  }
  // outputs
  for (int ai = 0; ai < na; ++ai) {
    for (int k = 0; k < 13; ++k) root_out[13 * ai + k] = root[13 * ai + k];
    if (E.actors[ai].fixed)
      for (int k = 7; k < 13; ++k) root_out[13 * ai + k] = 0.0;
  }
  for (int j = 0; j < nd; ++j) {
    dof_out[2 * j] = qj[j];
    dof_out[2 * j + 1] = qd[dcol[j]];
  }
  if (O.contact_force)
    for (int k = 0; k < 3 * E.n_bodies; ++k) O.contact_force[k] = cforce[k];
  if (O.contact_scale)
    for (int k = 0; k < 2 * E.n_bodies; ++k) O.contact_scale[k] = cscale[k];
  if (O.dof_force)
    for (int j = 0; j < nd; ++j) O.dof_force[j] = dforce[j] / P.substeps;
  if (O.mode) *O.mode = mode.h;
}

Params read_params(const double* p) {
  Params P;
  P.dt = p[ORC_P_DT];
  P.substeps = (int)p[ORC_P_SUBSTEPS];
  P.h = P.dt / P.substeps;
  P.g = {p[ORC_P_GX], p[ORC_P_GY], p[ORC_P_GZ]};
  P.iters = (int)p[ORC_P_ITERS];
  P.mu = p[ORC_P_MU];
  P.beta = p[ORC_P_BETA];
  P.mc = p[ORC_P_MC];
  P.ml_rev = p[ORC_P_ML_REV];
  P.ml_pri = p[ORC_P_ML_PRI];
  P.guard_c = p[ORC_P_GUARD_C];
  P.guard_l = p[ORC_P_GUARD_L];
  P.tgs = p[ORC_P_SOLVER] == 1.0 ? 1 : 0;
  return P;
}

}  // namespace

// ====================================================================== C API
extern "C" {

void orc_env_set_tendons(void* env, int n_tendons, const double* params, int n_joints, const double* joints) {
  Env& E = *static_cast<Env*>(env);
  E.tendons.assign(n_tendons, Tendon{});
  for (int t = 0; t < n_tendons; ++t) {
    const double* p = params + 6 * t;
    Tendon& T = E.tendons[t];
    T.k = p[0]; T.d = p[1]; T.rest = p[2]; T.lo = p[3]; T.hi = p[4]; T.klim = p[5];
  }
  for (int j = 0; j < n_joints; ++j) {
    const double* r = joints + 4 * j;
    Tendon& T = E.tendons[(int)r[0]];
    T.dof.push_back((int)r[1]);
    T.parent.push_back((int)r[2]);
    T.coef.push_back(r[3]);
  }
}

void* orc_env_create(int n_actors, int n_links, const double* links, int n_shapes, const double* shapes,
                     int n_pairs, const int* pairs, char* err, int errlen) {
  Env* E = new Env();
  std::string msg;
  E->actors.resize(n_actors);
  for (int i = 0; i < n_links; ++i) {
    const double* r = links + (size_t)i * ORC_L_COLS;
    int a = (int)r[ORC_L_ACTOR];
    if (a < 0 || a >= n_actors) { msg = "bad actor index in link table"; goto fail; }
    Link L;
    L.parent = (int)r[ORC_L_PARENT];
    L.jtype = (int)r[ORC_L_JOINT];
    L.anchor = {r[ORC_L_ANCHOR], r[ORC_L_ANCHOR + 1], r[ORC_L_ANCHOR + 2]};
    L.axis = {r[ORC_L_AXIS], r[ORC_L_AXIS + 1], r[ORC_L_AXIS + 2]};
    L.lo = r[ORC_L_LOWER]; L.hi = r[ORC_L_UPPER];
    L.kp = r[ORC_L_KP]; L.kd = r[ORC_L_KD]; L.armature = r[ORC_L_ARMATURE]; L.given_mass = r[ORC_L_MASS];
    double an = norm(L.axis);
    if (i > 0 && an > 0) L.axis = scl(L.axis, 1.0 / an);
    E->actors[a].links.push_back(L);
  }
  {
    std::vector<std::vector<int>> gmap(n_actors);  // global shape row -> actor-local index
    for (int i = 0; i < n_shapes; ++i) {
      const double* r = shapes + (size_t)i * ORC_S_COLS;
      int a = (int)r[ORC_S_ACTOR];
      if (a < 0 || a >= n_actors) { msg = "bad actor index in shape table"; goto fail; }
      Shape s;
      s.link = (int)r[ORC_S_LINK];
      s.kind = (int)r[ORC_S_KIND];
      s.p0 = {r[ORC_S_P0], r[ORC_S_P0 + 1], r[ORC_S_P0 + 2]};
      s.p1 = {r[ORC_S_P1], r[ORC_S_P1 + 1], r[ORC_S_P1 + 2]};
      s.r = r[ORC_S_RADIUS];
      s.half = {r[ORC_S_HALF], r[ORC_S_HALF + 1], r[ORC_S_HALF + 2]};
      s.density = r[ORC_S_DENSITY];
      Actor& A = E->actors[a];
      if (s.link < 0 || s.link >= (int)A.links.size()) { msg = "bad link index in shape table"; goto fail; }
      A.links[s.link].shapes.push_back((int)A.shapes.size());
      A.shapes.push_back(s);
    }
    int v_off = 0, dof_off = 0, body_off = 0;
    for (Actor& A : E->actors) {
      if (!compile_actor(A, msg)) goto fail;
      A.v_off = v_off; A.dof_off = dof_off; A.body_off = body_off;
      v_off += A.n_v; dof_off += A.n_dof; body_off += (int)A.links.size();
    }
    E->n_v = v_off; E->n_dof = dof_off; E->n_bodies = body_off;
    // pairs reference global shape rows; convert to actor-local indices
    std::vector<int> local(n_shapes), counter(n_actors, 0);
    for (int i = 0; i < n_shapes; ++i) local[i] = counter[(int)shapes[(size_t)i * ORC_S_COLS + ORC_S_ACTOR]]++;
    for (int i = 0; i < n_pairs; ++i) {
      const int* p = pairs + 6 * i;
      if (p[0] < 0 || p[0] >= n_actors || p[2] < 0 || p[2] >= n_shapes) { msg = "bad pair"; goto fail; }
      Pair P{p[0], p[1], local[p[2]], p[3], p[4], p[3] >= 0 ? local[p[5]] : -1};
      if (P.ba >= 0 && (P.ba >= n_actors || p[5] < 0 || p[5] >= n_shapes ||
                        E->actors[P.ba].shapes[P.bs].kind != S_BOX || E->actors[P.aa].shapes[P.as].kind == S_BOX)) {
        msg = "body-body pairs must be sphere/capsule vs box"; goto fail;
      }
      E->pairs.push_back(P);
    }
    int ns = 0;
    for (const Pair& P : E->pairs) ns += slots_of_pair(*E, P);
    E->n_slots = ns;
    int lim = 0;
    for (const Actor& A : E->actors)
      for (int j = 1; j < (int)A.links.size(); ++j)
        lim += std::isfinite(A.links[j].lo) + std::isfinite(A.links[j].hi);
    E->max_rows = lim + 3 * ns;
  }
  return E;
fail:
  if (err && errlen > 0) std::snprintf(err, errlen, "%s", msg.c_str());
  delete E;
  return nullptr;
}

void orc_env_destroy(void* env) { delete static_cast<Env*>(env); }

void orc_env_sizes(const void* env, int* out) {
  const Env* E = static_cast<const Env*>(env);
  out[0] = E->n_dof; out[1] = E->n_v; out[2] = E->n_bodies; out[3] = (int)E->actors.size();
  out[4] = E->max_rows; out[5] = E->n_slots;
}

void orc_mass_props(const void* env, double* mass, double* com, double* inertia) {
  const Env* E = static_cast<const Env*>(env);
  int b = 0;
  for (const Actor& A : E->actors)
    for (const Link& L : A.links) {
      mass[b] = L.m;
      for (int k = 0; k < 3; ++k) com[3 * b + k] = L.com[k];
      for (int k = 0; k < 9; ++k) inertia[9 * b + k] = L.Ic[k];
      ++b;
    }
}

void orc_fk(const void* env, const double* root_state, const double* dof_state, double* R, double* p) {
  const Env* E = static_cast<const Env*>(env);
  std::vector<double> qj, qd;
  split_state(*E, root_state, dof_state, qj, qd);
  for (size_t ai = 0; ai < E->actors.size(); ++ai) {
    const Actor& A = E->actors[ai];
    Kin K;
    kinematics(A, root_state + 13 * ai, &qj[A.dof_off], K);
    for (size_t i = 0; i < A.links.size(); ++i) {
      int b = A.body_off + (int)i;
      for (int k = 0; k < 9; ++k) R[9 * b + k] = K.R[i][k];
      for (int k = 0; k < 3; ++k) p[3 * b + k] = K.p[i][k];
    }
  }
}

void orc_body_states(const void* env, const double* root_state, const double* dof_state, double* out) {
  const Env* E = static_cast<const Env*>(env);
  std::vector<double> qj, qd;
  split_state(*E, root_state, dof_state, qj, qd);
  for (size_t ai = 0; ai < E->actors.size(); ++ai) {
    const Actor& A = E->actors[ai];
    Kin K;
    kinematics(A, root_state + 13 * ai, &qj[A.dof_off], K);
    const double* v = &qd[A.v_off];
    std::vector<v6> vel(A.links.size());
    for (size_t i = 0; i < A.links.size(); ++i) {
      const Link& L = A.links[i];
      if (i == 0) vel[0] = A.fixed ? v6{} : root_velocity(K.R[0], v);
      else vel[i] = v6add(m6v(K.X[i], vel[L.parent]), v6scl(K.S[i], v[L.col]));
      // link coordinates -> world: angular part and the linear velocity of the link origin
      const v3 w = mv(K.R[i], v3{vel[i][0], vel[i][1], vel[i][2]});
      const v3 u = mv(K.R[i], v3{vel[i][3], vel[i][4], vel[i][5]});
      double* o = out + 18 * (A.body_off + i);
      for (int k = 0; k < 3; ++k) o[k] = K.p[i][k];
      for (int k = 0; k < 9; ++k) o[3 + k] = K.R[i][k];
      for (int k = 0; k < 3; ++k) { o[12 + k] = u[k]; o[15 + k] = w[k]; }
    }
  }
}

int orc_dynamics(const void* env, const double* params, const double* root_state, const double* dof_state,
                 const double* tau, double* M, double* C, double* qdd_crba, double* qdd_aba) {
  const Env* E = static_cast<const Env*>(env);
  Params P = read_params(params);
  int nv = E->n_v;
  std::vector<double> qj, qd;
  split_state(*E, root_state, dof_state, qj, qd);
  std::vector<double> Mm(nv * nv, 0.0), Cc(nv, 0.0), zero(nv, 0.0), arm(nv, 0.0);
  for (size_t ai = 0; ai < E->actors.size(); ++ai) {
    const Actor& A = E->actors[ai];
    Kin K;
    kinematics(A, root_state + 13 * ai, &qj[A.dof_off], K);
    crba(A, K, &Mm[A.v_off * nv + A.v_off], nv);
    rnea(A, K, &qd[A.v_off], &zero[A.v_off], P.g, &Cc[A.v_off]);
    for (int j = 1; j < (int)A.links.size(); ++j) arm[A.v_off + A.links[j].col] = A.links[j].armature;
    if (qdd_aba) aba(A, K, &qd[A.v_off], &tau[A.v_off], &arm[A.v_off], P.g, &qdd_aba[A.v_off]);
  }
  if (M) std::copy(Mm.begin(), Mm.end(), M);
  if (C) std::copy(Cc.begin(), Cc.end(), C);
  if (qdd_crba) {
    std::vector<double> L = Mm;
    for (int c = 0; c < nv; ++c) L[c * nv + c] += arm[c];
    if (!cholesky(L, nv)) return -1;
    std::vector<double> x(nv);
    for (int c = 0; c < nv; ++c) x[c] = tau[c] - Cc[c];
    chol_solve(L, nv, x);
    std::copy(x.begin(), x.end(), qdd_crba);
  }
  return 0;
}

int orc_slots(const void* env, const double* root_state, const double* dof_state, double* phi, double* normal,
              double* point, int* body_a, int* body_b) {
  const Env* E = static_cast<const Env*>(env);
  std::vector<double> qj, qd;
  split_state(*E, root_state, dof_state, qj, qd);
  std::vector<Kin> K(E->actors.size());
  for (size_t ai = 0; ai < E->actors.size(); ++ai)
    kinematics(E->actors[ai], root_state + 13 * ai, &qj[E->actors[ai].dof_off], K[ai]);
  std::vector<Slot> slots;
  narrow_phase(*E, K, slots);
  for (size_t i = 0; i < slots.size(); ++i) {
    const Slot& s = slots[i];
    phi[i] = s.phi;
    for (int k = 0; k < 3; ++k) { normal[3 * i + k] = s.n[k]; point[3 * i + k] = s.x[k]; }
    body_a[i] = E->actors[s.a_actor].body_off + s.a_link;
    body_b[i] = s.b_actor >= 0 ? E->actors[s.b_actor].body_off + s.b_link : -1;
  }
  return (int)slots.size();
}

int orc_step(const void* env, const double* params, int n_envs, const double* root_in, const double* dof_in,
             const double* act, const double* pos_tgt, const double* vel_tgt, double* root_out, double* dof_out,
             double* qdd_free, int r_cap, int* row_count, int* row_key, double* row_lambda,
             double* contact_force, double* contact_scale, double* dof_force, int* near, unsigned long long* mode,
             int n_threads) {
  const Env* E = static_cast<const Env*>(env);
  if (!E || n_envs < 0 || !root_in || !dof_in || !act || !root_out || !dof_out) return -1;
  Params P = read_params(params);
  if (P.substeps < 1 || P.iters < 0 || !(P.dt > 0)) return -1;
  const int na = (int)E->actors.size(), nd = E->n_dof, nv = E->n_v, nb = E->n_bodies, S = P.substeps;
  std::vector<double> zeros(nd, 0.0);
  auto work = [&](int e0, int e1) {
    for (int e = e0; e < e1; ++e) {
      StepOut O;
      O.qdd_free = qdd_free ? qdd_free + (size_t)e * S * nv : nullptr;
      O.r_cap = r_cap;
      O.row_count = row_count ? row_count + (size_t)e * S : nullptr;
      O.row_key = row_key ? row_key + (size_t)e * S * r_cap : nullptr;
      O.row_lambda = row_lambda ? row_lambda + (size_t)e * S * r_cap : nullptr;
      O.contact_force = contact_force ? contact_force + (size_t)e * nb * 3 : nullptr;
      O.contact_scale = contact_scale ? contact_scale + (size_t)e * nb * 2 : nullptr;
      O.dof_force = dof_force ? dof_force + (size_t)e * nd : nullptr;
      O.near = near ? near + (size_t)e * S : nullptr;
      O.mode = mode ? mode + e : nullptr;
      step_env(*E, P, root_in + (size_t)e * na * 13, dof_in + (size_t)e * nd * 2, act + (size_t)e * nd,
               pos_tgt ? pos_tgt + (size_t)e * nd : zeros.data(), vel_tgt ? vel_tgt + (size_t)e * nd : zeros.data(),
               root_out + (size_t)e * na * 13, dof_out + (size_t)e * nd * 2, O);
    }
  };
  int T = std::max(1, std::min(n_threads, n_envs));
  if (T == 1) {
    work(0, n_envs);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back(work, (int)((long)n_envs * t / T), (int)((long)n_envs * (t + 1) / T));
    for (auto& x : th) x.join();
  }
  return 0;
}

}  // extern "C"
