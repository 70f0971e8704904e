// Host side of libags: model compilation, device tables, tensor binding and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ags.h"
#include "ags_internal.h"

using namespace ags;

namespace {
thread_local std::string g_err;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? AGS_E_NOMEM : AGS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- mass properties (closed forms)
struct Mass {
  double m = 0, c[3] = {0, 0, 0}, I[9] = {0};  // I about the COM, link frame
};

void add_outer(double* I, const double* a, const double* b, double s) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I[3 * i + j] += s * a[i] * b[j];
}

Mass shape_mass(const ags_shape_desc& s) {
  const double pi = 3.14159265358979323846;
  Mass r;
  double rho = s.density;
  if (s.kind == AGS_SHAPE_SPHERE) {
    double rad = s.radius;
    r.m = rho * 4.0 / 3.0 * pi * rad * rad * rad;
    for (int k = 0; k < 3; ++k) r.c[k] = s.p0[k];
    for (int k = 0; k < 3; ++k) r.I[4 * k] = 0.4 * r.m * rad * rad;
  } else if (s.kind == AGS_SHAPE_CAPSULE) {
    double d[3] = {double(s.p1[0]) - s.p0[0], double(s.p1[1]) - s.p0[1], double(s.p1[2]) - s.p0[2]};
    double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), rad = s.radius;
    double m_cyl = rho * pi * rad * rad * len;
    double m_caps = rho * 4.0 / 3.0 * pi * rad * rad * rad;
    r.m = m_cyl + m_caps;
    for (int k = 0; k < 3; ++k) r.c[k] = 0.5 * (double(s.p0[k]) + s.p1[k]);
    // axial: cylinder m r^2 / 2, caps (a full sphere) 2/5 m r^2; transverse: cylinder m (r^2/4 + L^2/12),
    // each cap about its own COM (3r/8 from its base) 83/320 m r^2, moved out to L/2 + 3r/8
    double ax = 0.5 * m_cyl * rad * rad + 0.4 * m_caps * rad * rad;
    double arm = 0.5 * len + 0.375 * rad;
    double tr = m_cyl * (rad * rad / 4.0 + len * len / 12.0) + m_caps * (83.0 / 320.0 * rad * rad + arm * arm);
    double u[3] = {0, 0, 1};
    if (len > 0)
      for (int k = 0; k < 3; ++k) u[k] = d[k] / len;
    for (int k = 0; k < 3; ++k) r.I[4 * k] = tr;
    add_outer(r.I, u, u, ax - tr);
  } else {
    double a = s.half[0], b = s.half[1], c = s.half[2];
    r.m = rho * 8.0 * a * b * c;
    for (int k = 0; k < 3; ++k) r.c[k] = s.p0[k];
    r.I[0] = r.m / 3.0 * (b * b + c * c);
    r.I[4] = r.m / 3.0 * (a * a + c * c);
    r.I[8] = r.m / 3.0 * (a * a + b * b);
  }
  return r;
}

Mass link_mass(const std::vector<const ags_shape_desc*>& shapes, double given) {
  Mass tot;
  std::vector<Mass> parts;
  for (auto* s : shapes) {
    parts.push_back(shape_mass(*s));
    tot.m += parts.back().m;
    for (int k = 0; k < 3; ++k) tot.c[k] += parts.back().m * parts.back().c[k];
  }
  if (tot.m > 0)
    for (int k = 0; k < 3; ++k) tot.c[k] /= tot.m;
  for (const Mass& p : parts) {
    double d[3] = {p.c[0] - tot.c[0], p.c[1] - tot.c[1], p.c[2] - tot.c[2]};
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    for (int k = 0; k < 9; ++k) tot.I[k] += p.I[k];
    for (int k = 0; k < 3; ++k) tot.I[4 * k] += p.m * dd;
    add_outer(tot.I, d, d, -p.m);
  }
  if (given > 0 && tot.m > 0) {
    double sc = given / tot.m;
    tot.m = given;
    for (int k = 0; k < 9; ++k) tot.I[k] *= sc;
  }
  return tot;
}
}  // namespace

struct ags_model {
  ags_model_info info{};
  int n_levels = 0, n_anc = 0;
  std::vector<int> li, level_begin, level_links, children, anc_link, dof_link, si, body_slot_begin, body_slot, ai;
  std::vector<double> lf, sf;
  std::vector<int> jtype;  // per link, to fill the limit margins at sim creation
  std::vector<unsigned long long> link_anc, col_anc;  // ancestor bit masks (links; generalized columns)
  std::vector<int> col_link;                           // owning link of each generalized column
  bool body_pairs = false;                             // has sphere/capsule-vs-box pairs
  int max_joint_entries = 0;  // most revolute/prismatic joints on the paths of one slot's two bodies
  std::vector<float> mass, com, inertia;
  // fixed tendons: per tendon joint (tendon, model DOF, model column, parent tendon joint or -1) and its
  // coefficient; per tendon stiffness, damping, rest length, lower, upper, limit stiffness
  std::vector<int> tj_i;
  std::vector<double> tj_f, tp;
  std::vector<int> actor_link_off;  // first link of each actor, then the link count
};

extern "C" const char* ags_last_error(void) { return g_err.c_str(); }

extern "C" int ags_model_add_tendons(ags_model* M, const ags_tendon_desc* T, int32_t n) {
  if (!M || n < 0 || (n > 0 && !T)) return fail(AGS_E_ARG, "tendons: bad arguments");
  std::vector<int> ti = M->tj_i;
  std::vector<double> tf = M->tj_f, tp = M->tp;
  for (int t = 0; t < n; ++t) {
    const ags_tendon_desc& d = T[t];
    if (d.actor < 0 || d.actor >= M->info.n_actors || d.n_joints <= 0 || !d.link || !d.parent || !d.coef)
      return fail(AGS_E_MODEL, "tendons: bad tendon description");
    const int tid = (int)tp.size() / 6, base = (int)tf.size();
    const int a = d.actor, lo = M->actor_link_off[a], hi = M->actor_link_off[a + 1];
    for (int j = 0; j < d.n_joints; ++j) {
      const int l = d.link[j], par = d.parent[j];
      if (l < 1 || lo + l >= hi || par < -1 || par >= j)
        return fail(AGS_E_MODEL, "tendons: link or parent out of range (parents first, no root links)");
      const int gl = lo + l;
      ti.insert(ti.end(), {tid, M->li[(size_t)gl * LI_COLS + LI_DOF], M->li[(size_t)gl * LI_COLS + LI_COL], par < 0 ? -1 : base + par});
      tf.push_back(d.coef[j]);
    }
    tp.insert(tp.end(), {d.stiffness, d.damping, d.rest_length, d.lower, d.upper, d.limit_stiffness});
  }
  M->tj_i = ti;
  M->tj_f = tf;
  M->tp = tp;
  return AGS_OK;
}

extern "C" int ags_model_create(const ags_actor_desc* actors, int32_t n_actors, const ags_pair_desc* pairs,
                                int32_t n_pairs, ags_model** out) {
  if (!actors || n_actors <= 0 || !out || (n_pairs > 0 && !pairs)) return fail(AGS_E_ARG, "model: bad arguments");
  *out = nullptr;
  ags_model* M = new ags_model();
  std::vector<int> link_off(n_actors), shape_off(n_actors);
  int nl = 0, ncol = 0, ndof = 0;
  M->ai.assign((size_t)n_actors * AI_COLS, 0);
  std::vector<int> depth;
  std::vector<std::vector<const ags_shape_desc*>> link_shapes;
  // links, columns, DOFs
  for (int a = 0; a < n_actors; ++a) {
    const ags_actor_desc& A = actors[a];
    if (A.n_links <= 0 || !A.links || (A.n_shapes > 0 && !A.shapes)) {
      delete M;
      return fail(AGS_E_MODEL, "model: actor without links");
    }
    link_off[a] = nl;
    const ags_link_desc& root = A.links[0];
    if (root.parent != -1 || (root.joint != AGS_JOINT_FREE && root.joint != AGS_JOINT_FIXED)) {
      delete M;
      return fail(AGS_E_MODEL, "model: the first link of an actor must be a free or fixed root");
    }
    const bool fixed = root.joint == AGS_JOINT_FIXED;
    M->ai[a * AI_COLS + AI_ROOT] = nl;
    M->ai[a * AI_COLS + AI_FIXED] = fixed;
    M->ai[a * AI_COLS + AI_COL] = fixed ? -1 : ncol;
    int rootcol = fixed ? -1 : ncol;
    if (!fixed) ncol += 6;
    for (int i = 0; i < A.n_links; ++i) {
      const ags_link_desc& L = A.links[i];
      if (i > 0 && (L.parent < 0 || L.parent >= i || (L.joint != AGS_JOINT_REVOLUTE && L.joint != AGS_JOINT_PRISMATIC))) {
        delete M;
        return fail(AGS_E_MODEL, "model: links must be in topological order with 1-DOF revolute/prismatic joints");
      }
      std::vector<int> row(LI_COLS, -1);
      std::vector<double> frow(LF_COLS, 0.0);
      row[LI_PARENT] = i == 0 ? -1 : link_off[a] + L.parent;
      row[LI_JTYPE] = L.joint;
      row[LI_ROOT] = link_off[a];
      row[LI_ROOTCOL] = rootcol;
      if (i == 0) {
        row[LI_COL] = rootcol;
        row[LI_DOF] = -1;
        depth.push_back(0);
      } else {
        row[LI_COL] = ncol++;
        row[LI_DOF] = ndof++;
        M->dof_link.push_back(nl);
        depth.push_back(depth[row[LI_PARENT]] + 1);
      }
      double an = std::sqrt(double(L.axis[0]) * L.axis[0] + double(L.axis[1]) * L.axis[1] + double(L.axis[2]) * L.axis[2]);
      for (int k = 0; k < 3; ++k) {
        frow[LF_ANCHOR + k] = L.anchor[k];
        frow[LF_AXIS + k] = (i > 0 && an > 0) ? L.axis[k] / an : L.axis[k];
      }
      if (i > 0 && !(an > 0)) {
        delete M;
        return fail(AGS_E_MODEL, "model: zero joint axis");
      }
      frow[LF_LO] = L.lower;
      frow[LF_HI] = L.upper;
      frow[LF_KP] = L.kp;
      frow[LF_KD] = L.kd;
      frow[LF_ARM] = L.armature;
      M->li.insert(M->li.end(), row.begin(), row.end());
      M->lf.insert(M->lf.end(), frow.begin(), frow.end());
      M->jtype.push_back(L.joint);
      link_shapes.emplace_back();
      ++nl;
    }
    for (int k = 0; k < A.n_shapes; ++k) {
      const ags_shape_desc& S = A.shapes[k];
      if (S.link < 0 || S.link >= A.n_links || S.kind < 0 || S.kind > 2) {
        delete M;
        return fail(AGS_E_MODEL, "model: bad shape");
      }
      link_shapes[link_off[a] + S.link].push_back(&S);
    }
  }
  if (nl > kMaxLinks || ncol > kMaxV) {
    delete M;
    return fail(AGS_E_ARG, "model: more than 64 links or 64 generalized velocities per environment");
  }
  // mass properties
  M->mass.resize(nl);
  M->com.resize(3 * nl);
  M->inertia.resize(9 * nl);
  {
    int g = 0;
    for (int a = 0; a < n_actors; ++a)
      for (int i = 0; i < actors[a].n_links; ++i, ++g) {
        Mass ms = link_mass(link_shapes[g], actors[a].links[i].mass);
        if (actors[a].links[i].mass > 0 && link_shapes[g].empty()) {
          delete M;
          return fail(AGS_E_MODEL, "model: a given link mass needs shapes for its distribution");
        }
        if (i == 0 && actors[a].links[0].joint == AGS_JOINT_FREE) {
          double cn = std::sqrt(ms.c[0] * ms.c[0] + ms.c[1] * ms.c[1] + ms.c[2] * ms.c[2]);
          if (cn > 1e-6 || ms.m <= 0) {
            delete M;
            return fail(AGS_E_MODEL, "model: a free root link must have mass and its frame at its centre of mass");
          }
        }
        double* fr = &M->lf[(size_t)g * LF_COLS];
        fr[LF_MASS] = ms.m;
        for (int k = 0; k < 3; ++k) fr[LF_COM + k] = ms.c[k];
        fr[LF_IC + 0] = ms.I[0];
        fr[LF_IC + 1] = ms.I[4];
        fr[LF_IC + 2] = ms.I[8];
        fr[LF_IC + 3] = 0.5 * (ms.I[1] + ms.I[3]);
        fr[LF_IC + 4] = 0.5 * (ms.I[2] + ms.I[6]);
        fr[LF_IC + 5] = 0.5 * (ms.I[5] + ms.I[7]);
        M->mass[g] = (float)ms.m;
        for (int k = 0; k < 3; ++k) M->com[3 * g + k] = (float)ms.c[k];
        for (int k = 0; k < 9; ++k) M->inertia[9 * g + k] = (float)ms.I[k];
      }
  }
  // every joint must carry inertia: a subtree without mass needs armature (its D would be 0)
  {
    std::vector<double> sub_mass(nl, 0.0);
    for (int i = nl - 1; i >= 0; --i) {
      sub_mass[i] += M->lf[(size_t)i * LF_COLS + LF_MASS];
      int p = M->li[i * LI_COLS + LI_PARENT];
      if (p >= 0) sub_mass[p] += sub_mass[i];
    }
    for (int i = 0; i < nl; ++i)
      if (M->li[i * LI_COLS + LI_PARENT] >= 0 && !(sub_mass[i] > 0) && !(M->lf[(size_t)i * LF_COLS + LF_ARM] > 0)) {
        delete M;
        return fail(AGS_E_MODEL, "model: a joint moves neither mass nor armature");
      }
  }
  // levels
  int maxd = 0;
  for (int d : depth) maxd = std::max(maxd, d);
  M->n_levels = maxd + 1;
  M->level_begin.assign(M->n_levels + 1, 0);
  for (int d = 0; d < M->n_levels; ++d) {
    M->level_begin[d] = (int)M->level_links.size();
    for (int i = 0; i < nl; ++i)
      if (depth[i] == d) M->level_links.push_back(i);
  }
  M->level_begin[M->n_levels] = nl;
  // children and non-root ancestors (CSR)
  for (int i = 0; i < nl; ++i) {
    M->li[i * LI_COLS + LI_CHILD_BEGIN] = (int)M->children.size();
    for (int c = i + 1; c < nl; ++c)
      if (M->li[c * LI_COLS + LI_PARENT] == i) M->children.push_back(c);
    M->li[i * LI_COLS + LI_CHILD_END] = (int)M->children.size();
    M->li[i * LI_COLS + LI_ANC_BEGIN] = (int)M->anc_link.size();
    std::vector<int> anc;
    int p = M->li[i * LI_COLS + LI_PARENT];
    while (p >= 0 && M->li[p * LI_COLS + LI_PARENT] >= 0) {
      anc.push_back(p);
      p = M->li[p * LI_COLS + LI_PARENT];
    }
    std::reverse(anc.begin(), anc.end());
    M->anc_link.insert(M->anc_link.end(), anc.begin(), anc.end());
    M->li[i * LI_COLS + LI_ANC_END] = (int)M->anc_link.size();
  }
  M->n_anc = (int)M->anc_link.size();
  // ancestor masks: links (ancestors and the link itself) and columns (columns preceding a column on
  // its path to the root: a free root's lower-numbered columns, then every column of its ancestors)
  M->link_anc.assign(nl, 0ull);
  M->col_link.assign(ncol, 0);
  M->col_anc.assign(ncol, 0ull);
  for (int i = 0; i < nl; ++i) {
    const int p = M->li[i * LI_COLS + LI_PARENT];
    M->link_anc[i] = (p >= 0 ? M->link_anc[p] : 0ull) | (1ull << i);
  }
  for (int i = 0; i < nl; ++i) {
    const int* row = &M->li[i * LI_COLS];
    std::vector<int> own;
    if (row[LI_PARENT] < 0) {
      if (row[LI_ROOTCOL] >= 0)
        for (int k = 0; k < 6; ++k) own.push_back(row[LI_ROOTCOL] + k);
    } else {
      own.push_back(row[LI_COL]);
    }
    unsigned long long above = 0ull;  // every column of the strict ancestors of link i
    for (int j = 0; j < nl; ++j) {
      if (j == i || !((M->link_anc[i] >> j) & 1ull)) continue;
      const int* rj = &M->li[j * LI_COLS];
      if (rj[LI_PARENT] < 0) {
        if (rj[LI_ROOTCOL] >= 0)
          for (int k = 0; k < 6; ++k) above |= 1ull << (rj[LI_ROOTCOL] + k);
      } else {
        above |= 1ull << rj[LI_COL];
      }
    }
    for (size_t a = 0; a < own.size(); ++a) {
      M->col_link[own[a]] = i;
      unsigned long long m = above;
      for (size_t b = 0; b < a; ++b) m |= 1ull << own[b];
      M->col_anc[own[a]] = m;
    }
  }
  // contact slots: plane pairs (sphere 1, capsule 2 caps, box 8 corners); box pairs (sphere 1, capsule 2 caps + midpoint)
  std::vector<std::vector<int>> body_entries(nl);
  int limited = 0;
  for (int i = 0; i < nl; ++i)
    if (M->jtype[i] == AGS_JOINT_REVOLUTE || M->jtype[i] == AGS_JOINT_PRISMATIC)
      limited += std::isfinite(M->lf[i * LF_COLS + LF_LO]) + std::isfinite(M->lf[i * LF_COLS + LF_HI]);
  for (int p = 0; p < n_pairs; ++p) {
    const ags_pair_desc& P = pairs[p];
    if (P.a_actor < 0 || P.a_actor >= n_actors || P.a_shape < 0 || P.a_shape >= actors[P.a_actor].n_shapes ||
        P.b_actor >= n_actors || (P.b_actor >= 0 && (P.b_shape < 0 || P.b_shape >= actors[P.b_actor].n_shapes))) {
      delete M;
      return fail(AGS_E_MODEL, "model: bad pair");
    }
    const ags_shape_desc& A = actors[P.a_actor].shapes[P.a_shape];
    const int ka = link_off[P.a_actor] + A.link;
    std::vector<std::vector<double>> pts;  // sphere centres or corners in link a's frame
    int type;
    int kb = -1;
    const ags_shape_desc* B = nullptr;
    if (P.b_actor < 0) {
      if (A.kind == AGS_SHAPE_BOX) {
        type = SLOT_CORNER_PLANE;
        for (int c = 0; c < 8; ++c)
          pts.push_back({double(A.p0[0]) + ((c & 1) ? A.half[0] : -A.half[0]),
                         double(A.p0[1]) + ((c & 2) ? A.half[1] : -A.half[1]),
                         double(A.p0[2]) + ((c & 4) ? A.half[2] : -A.half[2])});
      } else {
        type = SLOT_SPHERE_PLANE;
        pts.push_back({A.p0[0], A.p0[1], A.p0[2]});
        if (A.kind == AGS_SHAPE_CAPSULE) pts.push_back({A.p1[0], A.p1[1], A.p1[2]});
      }
    } else {
      B = &actors[P.b_actor].shapes[P.b_shape];
      if (B->kind != AGS_SHAPE_BOX || A.kind == AGS_SHAPE_BOX || P.b_actor == P.a_actor) {
        delete M;
        return fail(AGS_E_MODEL, "model: body pairs must be a sphere or capsule against a box of another actor");
      }
      type = SLOT_SPHERE_BOX;
      M->body_pairs = true;
      kb = link_off[P.b_actor] + B->link;
      pts.push_back({A.p0[0], A.p0[1], A.p0[2]});
      if (A.kind == AGS_SHAPE_CAPSULE) {
        pts.push_back({A.p1[0], A.p1[1], A.p1[2]});
        pts.push_back({0.5 * (double(A.p0[0]) + A.p1[0]), 0.5 * (double(A.p0[1]) + A.p1[1]),
                       0.5 * (double(A.p0[2]) + A.p1[2])});
      }
    }
    for (size_t k = 0; k < pts.size(); ++k) {
      int slot = (int)(M->si.size() / SI_COLS);
      M->si.insert(M->si.end(), {type, ka, kb, (p << 8) | (int)k});
      std::vector<double> f(SF_COLS, 0.0);
      for (int q = 0; q < 3; ++q) f[SF_P + q] = pts[k][q];
      f[SF_R] = type == SLOT_CORNER_PLANE ? 0.0 : A.radius;
      if (B)
        for (int q = 0; q < 3; ++q) {
          f[SF_BOXC + q] = B->p0[q];
          f[SF_HALF + q] = B->half[q];
        }
      M->sf.insert(M->sf.end(), f.begin(), f.end());
      body_entries[ka].push_back(2 * slot);
      if (kb >= 0) body_entries[kb].push_back(2 * slot + 1);
    }
  }
  const int ns = (int)(M->si.size() / SI_COLS);
  {
    auto joints_to_root = [&](int k) {
      int n = 0;
      for (; k >= 0; k = M->li[k * LI_COLS + LI_PARENT])
        n += M->jtype[k] == AGS_JOINT_REVOLUTE || M->jtype[k] == AGS_JOINT_PRISMATIC;
      return n;
    };
    for (int sl = 0; sl < ns; ++sl) {
      const int* r = &M->si[(size_t)sl * SI_COLS];
      M->max_joint_entries = std::max(M->max_joint_entries,
                                      joints_to_root(r[SI_LINK_A]) + (r[SI_LINK_B] >= 0 ? joints_to_root(r[SI_LINK_B]) : 0));
    }
  }
  if (ns > kMaxSlots) {
    delete M;
    return fail(AGS_E_ARG, "model: more than 256 contact slots per environment");
  }
  M->body_slot_begin.assign(nl + 1, 0);
  for (int i = 0; i < nl; ++i) {
    M->body_slot_begin[i] = (int)M->body_slot.size();
    M->body_slot.insert(M->body_slot.end(), body_entries[i].begin(), body_entries[i].end());
  }
  M->body_slot_begin[nl] = (int)M->body_slot.size();
  M->info.n_actors = n_actors;
  M->actor_link_off.assign(link_off.begin(), link_off.end());
  M->actor_link_off.push_back(nl);
  M->info.n_links = nl;
  M->info.n_dof = ndof;
  M->info.n_v = ncol;
  M->info.n_slots = ns;
  M->info.max_rows = limited + 3 * ns;
  *out = M;
  return AGS_OK;
}

extern "C" void ags_model_destroy(ags_model* m) { delete m; }

extern "C" int ags_model_get_info(const ags_model* m, ags_model_info* out) {
  if (!m || !out) return fail(AGS_E_ARG, "bad arguments");
  *out = m->info;
  return AGS_OK;
}

extern "C" int ags_model_mass_props(const ags_model* m, float* mass, float* com, float* inertia) {
  if (!m) return fail(AGS_E_ARG, "bad arguments");
  if (mass) std::copy(m->mass.begin(), m->mass.end(), mass);
  if (com) std::copy(m->com.begin(), m->com.end(), com);
  if (inertia) std::copy(m->inertia.begin(), m->inertia.end(), inertia);
  return AGS_OK;
}

// ---------------------------------------------------------------- simulation
namespace {
struct TypeDev {
  int model = 0;  // index of the model among those the sim was created with
  int team = 64;
  DevModel dm{};
  Lds lds{};
  void* block = nullptr;       // device tables
  int* env_list = nullptr;     // device env ids of this type
  // per-type launches with one environment per wavefront: the env ids in the order the next step dispatches
  // them (most rows in the previous step first), and the reordering's buffer
  int* step_order = nullptr;
  int* order_tmp = nullptr;
  int n_envs = 0;
  void* scratch = nullptr;
  long long scratch_stride = 0;  // elements of the compute type per env
  AdjLds adj{};
  size_t adj_bytes = 0;           // LDS of the adjoint kernel
  AdjLds adj_small{};             // the same with at most kAdjSmallRows rows (first pass of a two-pass adjoint)
  size_t adj_small_bytes = 0;
  bool adj_two = false;           // rows may exceed kAdjSmallRows: small layout first, overflow retried
  bool body_pairs = false;
};

int adj_fp64(const ags_sim_params& p) { return p.adjoint_precision == 64 || (p.adjoint_precision == 0 && p.compute_fp64); }

Lds make_layout(const ags_model_info& info, int n_levels, int n_anc, int team, size_t elem) {
  Lds L{};
  int off = 0;
  const int ratio = (int)(elem / sizeof(int));  // ints per compute-type word
  auto take = [&](int words) {
    int o = off;
    off += (std::max(words, 1) + 1) & ~1;  // keep 8-byte alignment of every array
    return o;
  };
  auto take_i = [&](int ints) { return take((ints + ratio - 1) / ratio); };
  const int nl = info.n_links, na = info.n_actors, nd = info.n_dof, nv = info.n_v, ns = info.n_slots;
  const int rc = std::max(1, info.max_rows);
  // integer model tables, shared by the environments of a workgroup
  L.t_li = take_i(nl * LI_COLS); L.t_lev = take_i(n_levels + 1); L.t_links = take_i(nl);
  L.t_child = take_i(nl); L.t_anc = take_i(n_anc); L.t_dof = take_i(nd); L.t_ai = take_i(na * AI_COLS);
  L.team_base = off;
  // per environment, offsets relative to its region
  off = 0;
  L.qj = take(nd); L.qd = take(nv); L.root = take(13 * na); L.F = take(3 * nl);
  L.L0 = take(27 * na); L.vs = take(nv);
  L.o = take(3 * nl); L.ax = take(3 * nl); L.U = take(6 * nl); L.Dinv = take(nl); L.Ubar = take(3 * nl);
  L.G = take(n_anc);
  L.phi = take(ns); L.n = take(3 * ns); L.x = take(3 * ns); L.sact = take_i(ns);
  L.rkr = take_i(rc); L.rbias = take(rc); L.rinvA = take(rc); L.rlam = take(rc);
  L.misc = take_i(8);
  // the dynamics arrays (forward sweep to narrow phase) and the row-response chunks are never live together
  const int shared = off;
  L.q = take(4 * nl); L.v = take(6 * nl); L.IA = take(21 * nl); L.pA = take(6 * nl); L.u = take(nl);
  L.tau = take(nv); L.arm = take(nv);
  const int dyn_end = off;
  off = shared;
  L.wstride = nv | 1;
  L.W = take(kFastRows * L.wstride);
  off = std::max(off, dyn_end);
  L.team_stride = off;
  L.total = L.team_base + (kTeam / team) * L.team_stride;
  return L;
}
}  // namespace

// Scratch of ags_rollout_backward_noalloc: its two segment buffers live in this array instead of a
// caller-owned workspace.  Every device the library runs on holds its own copy until the process ends.  In
// host code `scratch` only names the symbol; the device address of the current device's copy comes from
// hipGetSymbolAddress, taken once per device when a sim is created there (noalloc_scratch_ptr).
constexpr long long kNoAllocScratchBytes = 64ll << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// this device's copy of `scratch` (looked up on the first call on each device)
hipError_t noalloc_scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

struct ags_sim {
  ags_sim_params params{};
  int n_envs = 0;
  std::vector<TypeDev> types;
  std::vector<int> env_model;
  int* env_tables = nullptr;  // device: actor base, dof base, body base (3 x n_envs)
  int* actor_rows = nullptr;  // device: root row begin, root count(1), dof begin, dof count (4 x N_A)
  int n_actors_total = 0, n_dof_total = 0, n_bodies_total = 0, max_nv = 0, max_rows = 0;
  void* bound[AGS_NUM_TENSORS] = {nullptr};
  float* kp_dof = nullptr;  // device: drive stiffness of every DOF (target adjoints)
  double* mid_root = nullptr;  // set while a rollout recomputes: where the step writes substep states
  int* adj_retry = nullptr;    // device: count, then the environments the small adjoint layout could not hold
  int* adj_big_list = nullptr; // device: count, then the flagged environments of the current type
  int* env_rows = nullptr;     // device: most rows of a substep in each env's last step (dispatch order)
  int n_cu = 1;                // compute units of the sim's device
  // rollout backward: a second stream (default priority) recomputes the next segment while the adjoint of
  // the current one runs; events order the two segment buffers between the streams
  hipStream_t aux = nullptr;
  hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  // the forward flags environments with many rows (big_out, per step); their adjoints then run with the full
  // layout on a third stream beside the small-layout pass (adj_big: this step's flags, or none)
  int* big_out = nullptr;
  const int* adj_big = nullptr;
  // set while a rollout reverses its steps: the adjoint writes only failures into the status array, which the
  // rollout cleared first, so an env over the row capacity at any step stays flagged
  int adj_sticky = 0;
  // device address of this device's copy of the no-allocation rollout scratch (see noalloc_scratch_ptr)
  void* noalloc_scratch = nullptr;
  hipStream_t aux2 = nullptr;
  hipEvent_t ev_big_start = nullptr, ev_big_done = nullptr, ev_big_listed = nullptr;
  // persistent (fused) launch
  bool fused_ok = false;
  int* units = nullptr;  // device: (type, group) pairs
  int n_units = 0, fused_grid = 0, fused_team = 64;
  size_t fused_lds = 0;
};

namespace {
hipError_t ensure_streams(ags_sim* S);
}

extern "C" int ags_sim_create(const ags_model* const* models, int32_t n_models, const int32_t* env_model,
                              int32_t n_envs, const ags_sim_params* p, ags_sim** out) {
  if (!models || n_models <= 0 || !env_model || n_envs <= 0 || !p || !out) return fail(AGS_E_ARG, "sim: bad arguments");
  if (!(p->dt > 0) || p->substeps < 1 || p->pgs_iters < 0) return fail(AGS_E_ARG, "sim: bad parameters");
  if (p->adjoint_precision != 0 && p->adjoint_precision != 32 && p->adjoint_precision != 64)
    return fail(AGS_E_ARG, "sim: adjoint_precision must be 0, 32 or 64");
  if (p->adjoint_max_rows < 0 || p->adjoint_max_rows > kAdjRows)
    return fail(AGS_E_ARG, "sim: adjoint_max_rows must be 0 (default 64) or 1..64");
  if (p->solver != AGS_SOLVER_PGS && p->solver != AGS_SOLVER_TGS) return fail(AGS_E_ARG, "sim: unknown solver");
  *out = nullptr;
  for (int e = 0; e < n_envs; ++e)
    if (env_model[e] < 0 || env_model[e] >= n_models || !models[env_model[e]])
      return fail(AGS_E_ARG, "sim: bad env model index");
  ags_sim* S = new ags_sim();
  S->params = *p;
  S->n_envs = n_envs;
  S->env_model.assign(env_model, env_model + n_envs);
  std::vector<int> tables(3 * (size_t)n_envs), rows;
  std::vector<std::vector<int>> lists(n_models);
  int ab = 0, db = 0, bb = 0;
  for (int e = 0; e < n_envs; ++e) {
    const ags_model* M = models[env_model[e]];
    tables[e] = ab;
    tables[n_envs + e] = db;
    tables[2 * n_envs + e] = bb;
    int d = db;
    for (int a = 0; a < M->info.n_actors; ++a) {
      int root = M->ai[a * AI_COLS + AI_ROOT];
      int next_root = a + 1 < M->info.n_actors ? M->ai[(a + 1) * AI_COLS + AI_ROOT] : M->info.n_links;
      int nd = next_root - root - 1;
      rows.insert(rows.end(), {ab + a, 1, d, nd});
      d += nd;
    }
    lists[env_model[e]].push_back(e);
    ab += M->info.n_actors;
    db += M->info.n_dof;
    bb += M->info.n_links;
    S->max_nv = std::max(S->max_nv, M->info.n_v);
    S->max_rows = std::max(S->max_rows, M->info.max_rows);
  }
  S->n_actors_total = ab;
  S->n_dof_total = db;
  S->n_bodies_total = bb;
  hipError_t err;
  if ((err = hipMalloc(&S->env_tables, tables.size() * sizeof(int))) != hipSuccess ||
      (err = hipMemcpy(S->env_tables, tables.data(), tables.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMalloc(&S->actor_rows, rows.size() * sizeof(int))) != hipSuccess ||
      (err = hipMemcpy(S->actor_rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) {
    ags_sim_destroy(S);
    return hip_fail(err, "sim: upload");
  }
  {
    std::vector<float> kp(std::max(1, S->n_dof_total), 0.f);
    for (int e = 0, d = 0; e < n_envs; ++e) {
      const ags_model* M = models[env_model[e]];
      for (int j = 0; j < M->info.n_dof; ++j)
        kp[d + j] = (float)M->lf[(size_t)M->dof_link[j] * LF_COLS + LF_KP];
      d += M->info.n_dof;
    }
    if ((err = hipMalloc(&S->kp_dof, kp.size() * sizeof(float))) != hipSuccess ||
        (err = hipMemcpy(S->kp_dof, kp.data(), kp.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
      ags_sim_destroy(S);
      return hip_fail(err, "sim: drive table");
    }
  }
  const size_t elem_size = p->compute_fp64 ? sizeof(double) : sizeof(float);
  int max_type_envs = 0;
  for (int t = 0; t < n_models; ++t) {
    if (lists[t].empty()) continue;
    const ags_model* M = models[t];
    TypeDev T;
    T.model = t;
    T.n_envs = (int)lists[t].size();
    // lanes per environment: 64 unless 32 (two environments per wavefront) is asked for and every per-lane
    // loop fits; the 64-lane form has the wide row path, the dispatch order by rows and the inward sweep by
    // matrix entry, and is the faster one for both precisions on the humanoid-like workload
    T.team = p->lanes_per_env == 32 && M->info.n_v <= 32 ? 32 : 64;
    if (p->persistent) {  // one lane count for all types: 32 only if asked for and every type fits
      bool all32 = p->lanes_per_env == 32;
      for (int u = 0; u < n_models; ++u)
        if (!lists[u].empty() && models[u]->info.n_v > 32) all32 = false;
      T.team = all32 ? 32 : 64;
    }
    T.lds = make_layout(M->info, M->n_levels, M->n_anc, T.team, elem_size);
    // limit margins per joint type
    std::vector<double> lf = M->lf;
    for (int i = 0; i < M->info.n_links; ++i)
      lf[i * LF_COLS + LF_ML] = M->jtype[i] == AGS_JOINT_PRISMATIC ? p->limit_margin_pri : p->limit_margin_rev;
    // one device block: ints then floats
    std::vector<std::pair<const void*, size_t>> parts = {
        {M->li.data(), M->li.size() * 4}, {M->level_begin.data(), M->level_begin.size() * 4},
        {M->level_links.data(), M->level_links.size() * 4}, {M->children.data(), M->children.size() * 4},
        {M->anc_link.data(), M->anc_link.size() * 4}, {M->dof_link.data(), M->dof_link.size() * 4},
        {M->si.data(), M->si.size() * 4}, {M->body_slot_begin.data(), M->body_slot_begin.size() * 4},
        {M->body_slot.data(), M->body_slot.size() * 4}, {M->ai.data(), M->ai.size() * 4},
        {lists[t].data(), lists[t].size() * 4}, {lf.data(), lf.size() * 8}, {M->sf.data(), M->sf.size() * 8},
        {M->link_anc.data(), M->link_anc.size() * 8}, {M->col_anc.data(), M->col_anc.size() * 8},
        {M->col_link.data(), M->col_link.size() * 4}, {M->tj_i.data(), M->tj_i.size() * 4},
        {M->tj_f.data(), M->tj_f.size() * 8}, {M->tp.data(), M->tp.size() * 8}};
    size_t total = 0;
    std::vector<size_t> offs;
    for (auto& q : parts) {
      offs.push_back(total);
      total += (q.second + 255) & ~size_t(255);
    }
    if ((err = hipMalloc(&T.block, std::max<size_t>(total, 256))) != hipSuccess) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return hip_fail(err, "sim: model tables");
    }
    std::vector<char> host(total, 0);
    for (size_t k = 0; k < parts.size(); ++k)
      if (parts[k].second) std::memcpy(host.data() + offs[k], parts[k].first, parts[k].second);
    if ((err = hipMemcpy(T.block, host.data(), total, hipMemcpyHostToDevice)) != hipSuccess) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return hip_fail(err, "sim: model upload");
    }
    char* b = static_cast<char*>(T.block);
    DevModel& D = T.dm;
    D.n_links = M->info.n_links;
    D.n_actors = M->info.n_actors;
    D.n_dof = M->info.n_dof;
    D.n_v = M->info.n_v;
    D.n_slots = M->info.n_slots;
    D.n_levels = M->n_levels;
    D.n_anc = M->n_anc;
    D.r_cap = std::max(1, M->info.max_rows);
    D.n_body_slot = (int)M->body_slot.size();
    D.jfast = M->max_joint_entries <= kJointEntries;
    D.li = (const int*)(b + offs[0]);
    D.level_begin = (const int*)(b + offs[1]);
    D.level_links = (const int*)(b + offs[2]);
    D.children = (const int*)(b + offs[3]);
    D.anc_link = (const int*)(b + offs[4]);
    D.dof_link = (const int*)(b + offs[5]);
    D.si = (const int*)(b + offs[6]);
    D.body_slot_begin = (const int*)(b + offs[7]);
    D.body_slot = (const int*)(b + offs[8]);
    D.ai = (const int*)(b + offs[9]);
    T.env_list = (int*)(b + offs[10]);
    D.lf = (const double*)(b + offs[11]);
    D.sf = (const double*)(b + offs[12]);
    D.link_anc = (const unsigned long long*)(b + offs[13]);
    D.col_anc = (const unsigned long long*)(b + offs[14]);
    D.col_link = (const int*)(b + offs[15]);
    D.n_tj = (int)M->tj_f.size();
    D.tj_i = (const int*)(b + offs[16]);
    D.tj_f = (const double*)(b + offs[17]);
    D.tp = (const double*)(b + offs[18]);
    T.body_pairs = M->body_pairs;
    const int adj_cap = p->adjoint_max_rows > 0 ? p->adjoint_max_rows : kAdjRows;
    const int adj_small_cap = std::min(adj_cap, kAdjSmallRows);
    T.adj = make_adj_layout(M->info, p->substeps, std::min(p->pgs_iters, kAdjIters), adj_cap, adj_fp64(*p));
    T.adj_bytes = (size_t)T.adj.n_real * (adj_fp64(*p) ? sizeof(double) : sizeof(float)) + (size_t)T.adj.n_int * sizeof(int);
    T.adj_two = std::min(M->info.max_rows, adj_cap) > adj_small_cap;
    T.adj_small = make_adj_layout(M->info, p->substeps, std::min(p->pgs_iters, kAdjIters), adj_small_cap, adj_fp64(*p));
    T.adj_small_bytes = (size_t)T.adj_small.n_real * (adj_fp64(*p) ? sizeof(double) : sizeof(float)) +
                        (size_t)T.adj_small.n_int * sizeof(int);
    max_type_envs = std::max(max_type_envs, T.n_envs);
    if (T.adj_bytes <= 160 * 1024 && T.adj_bytes > 64 * 1024 &&
        (err = set_adjoint_lds_limit(adj_fp64(*p), T.adj_bytes)) != hipSuccess) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return hip_fail(err, "sim: adjoint LDS limit");
    }
    // J and W rows (slow path), then the wide path's columns of A (one entry per lane of a 64-lane team)
    T.scratch_stride = 2ll * D.r_cap * std::max(1, D.n_v) + (T.team == 64 ? 64ll * 64 : 0);
    T.scratch_stride = (T.scratch_stride + 63) & ~63ll;
    if (T.team == 64) {
      if ((err = hipMalloc(&T.step_order, 2 * sizeof(int) * T.n_envs)) != hipSuccess ||
          (err = hipMemcpy(T.step_order, lists[t].data(), sizeof(int) * T.n_envs, hipMemcpyHostToDevice)) != hipSuccess) {
        S->types.push_back(T);
        ags_sim_destroy(S);
        return hip_fail(err, "sim: dispatch order");
      }
      T.order_tmp = T.step_order + T.n_envs;
    }
    const size_t elem = p->compute_fp64 ? sizeof(double) : sizeof(float);
    const int epw = kTeam / T.team;
    const size_t padded = (size_t)((T.n_envs + epw - 1) / epw) * epw;
    if ((err = hipMalloc(&T.scratch, (size_t)T.scratch_stride * padded * elem)) != hipSuccess) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return hip_fail(err, "sim: scratch");
    }
    const size_t lds_bytes = (size_t)T.lds.total * elem;
    if (lds_bytes > 160 * 1024) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return fail(AGS_E_ARG, "sim: model too large for one workgroup's LDS");
    }
    if (lds_bytes > 64 * 1024 && (err = set_lds_limit(p->compute_fp64, T.team, lds_bytes)) != hipSuccess) {
      S->types.push_back(T);
      ags_sim_destroy(S);
      return hip_fail(err, "sim: LDS limit");
    }
    S->types.push_back(T);
  }
  int dev_cu = 0, n_cu = 0;
  if ((err = hipMalloc(&S->env_rows, (size_t)S->n_envs * sizeof(int))) != hipSuccess ||
      (err = hipMemset(S->env_rows, 0, (size_t)S->n_envs * sizeof(int))) != hipSuccess ||
      (err = hipMalloc(&S->adj_retry, ((size_t)max_type_envs + 1) * sizeof(int))) != hipSuccess ||
      (err = hipMalloc(&S->adj_big_list, ((size_t)max_type_envs + 1) * sizeof(int))) != hipSuccess ||
      (err = hipGetDevice(&dev_cu)) != hipSuccess ||
      (err = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_cu)) != hipSuccess) {
    ags_sim_destroy(S);
    return hip_fail(err, "sim: adjoint lists");
  }
  S->n_cu = std::max(1, n_cu);
  // the rollout streams and this device's no-allocation scratch are set up here, so that no rollout call
  // creates or looks up anything
  if ((err = ensure_streams(S)) != hipSuccess || (err = noalloc_scratch_ptr(dev_cu, &S->noalloc_scratch)) != hipSuccess) {
    ags_sim_destroy(S);
    return hip_fail(err, "sim: rollout streams / scratch");
  }
  if (p->persistent && !S->types.empty() && (int)S->types.size() <= kMaxFusedTypes) {
    // work list: (type, group) units, types ordered by estimated cost per group (heaviest first)
    std::vector<int> order(S->types.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    auto cost = [&](const TypeDev& T) {
      const double nv = T.dm.n_v;
      return (nv * nv + 4.0 * T.dm.n_slots + 8.0 * T.dm.n_links) * (kTeam / T.team);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(S->types[a]) > cost(S->types[b]); });
    std::vector<int> units;
    size_t lds_words = 0;
    for (int k : order) {
      const TypeDev& T = S->types[k];
      const int epw = kTeam / T.team;
      const int groups = (T.n_envs + epw - 1) / epw;
      for (int g = 0; g < groups; ++g) units.insert(units.end(), {k, g});
      lds_words = std::max(lds_words, (size_t)T.lds.total);
    }
    S->fused_team = S->types[0].team;
    S->fused_lds = lds_words * elem_size;
    S->n_units = (int)(units.size() / 2);
    int dev = 0, cus = 0, per_cu = 0;
    if (S->fused_lds <= 160 * 1024 &&
        (err = hipGetDevice(&dev)) == hipSuccess &&
        (err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) == hipSuccess &&
        (S->fused_lds <= 64 * 1024 || (err = set_fused_lds_limit(p->compute_fp64, S->fused_team, S->fused_lds)) == hipSuccess) &&
        (err = fused_blocks_per_cu(p->compute_fp64, S->fused_team, S->fused_lds, &per_cu)) == hipSuccess &&
        (err = hipMalloc(&S->units, units.size() * sizeof(int))) == hipSuccess &&
        (err = hipMemcpy(S->units, units.data(), units.size() * sizeof(int), hipMemcpyHostToDevice)) == hipSuccess) {
      S->fused_grid = std::max(1, std::min(S->n_units, cus * std::max(1, per_cu)));
      S->fused_ok = true;
    } else {
      ags_sim_destroy(S);
      return err != hipSuccess ? hip_fail(err, "sim: persistent launch set-up")
                               : fail(AGS_E_ARG, "sim: environment types too large for one persistent launch");
    }
  } else if (p->persistent) {
    ags_sim_destroy(S);
    return fail(AGS_E_ARG, "sim: a persistent launch takes at most 4 environment types");
  }
  *out = S;
  return AGS_OK;
}

extern "C" void ags_sim_destroy(ags_sim* S) {
  if (!S) return;
  for (TypeDev& T : S->types) {
    if (T.block) (void)hipFree(T.block);
    if (T.scratch) (void)hipFree(T.scratch);
    if (T.step_order) (void)hipFree(T.step_order);
  }
  if (S->adj_retry) (void)hipFree(S->adj_retry);
  if (S->env_rows) (void)hipFree(S->env_rows);
  if (S->adj_big_list) (void)hipFree(S->adj_big_list);
  for (int k = 0; k < 2; ++k) {
    if (S->ev_ready[k]) (void)hipEventDestroy(S->ev_ready[k]);
    if (S->ev_free[k]) (void)hipEventDestroy(S->ev_free[k]);
  }
  if (S->aux) (void)hipStreamDestroy(S->aux);
  if (S->ev_big_start) (void)hipEventDestroy(S->ev_big_start);
  if (S->ev_big_done) (void)hipEventDestroy(S->ev_big_done);
  if (S->ev_big_listed) (void)hipEventDestroy(S->ev_big_listed);
  if (S->aux2) (void)hipStreamDestroy(S->aux2);
  if (S->env_tables) (void)hipFree(S->env_tables);
  if (S->units) (void)hipFree(S->units);
  if (S->kp_dof) (void)hipFree(S->kp_dof);
  if (S->actor_rows) (void)hipFree(S->actor_rows);
  delete S;
}

extern "C" int ags_sim_tensor_shape(const ags_sim* S, int32_t which, int64_t* rows, int64_t* cols) {
  if (!S || !rows || !cols) return fail(AGS_E_ARG, "bad arguments");
  const int sub = S->params.substeps;
  switch (which) {
    case AGS_ROOT_STATE: *rows = S->n_actors_total; *cols = 13; break;
    case AGS_DOF_STATE: *rows = S->n_dof_total; *cols = 2; break;
    case AGS_DOF_ACTUATION: case AGS_DOF_POS_TARGET: case AGS_DOF_VEL_TARGET: case AGS_DOF_FORCE:
      *rows = S->n_dof_total; *cols = 1; break;
    case AGS_NET_CONTACT_FORCE: *rows = S->n_bodies_total; *cols = 3; break;
    case AGS_RIGID_BODY_STATE: *rows = S->n_bodies_total; *cols = 13; break;
    case AGS_ENV_STATUS: *rows = S->n_envs; *cols = 1; break;
    case AGS_BODY_MASS_SCALE: *rows = S->n_bodies_total; *cols = 1; break;
    case AGS_DOF_STIFFNESS: case AGS_DOF_DAMPING: *rows = S->n_dof_total; *cols = 1; break;
    case AGS_DOF_LIMITS: *rows = S->n_dof_total; *cols = 2; break;
    case AGS_ENV_FRICTION: *rows = S->n_envs; *cols = 1; break;
    case AGS_ENV_GRAVITY: *rows = S->n_envs; *cols = 3; break;
    case AGS_DEBUG_QDD_FREE: *rows = S->n_envs; *cols = (int64_t)sub * S->max_nv; break;
    case AGS_DEBUG_ROW_COUNT: *rows = S->n_envs; *cols = sub; break;
    case AGS_DEBUG_ROW_KEY: case AGS_DEBUG_ROW_LAMBDA: *rows = S->n_envs; *cols = (int64_t)sub * std::max(1, S->max_rows); break;
    case AGS_DEBUG_PHASE_CYCLES: *rows = S->n_envs; *cols = kPhases; break;
    case AGS_DEBUG_ADJ_CYCLES: *rows = S->n_envs; *cols = kAdjPhases; break;
    default: return fail(AGS_E_ARG, "unknown tensor");
  }
  return AGS_OK;
}

extern "C" int ags_sim_bind(ags_sim* S, int32_t which, void* ptr) {
  if (!S || which < 0 || which >= AGS_NUM_TENSORS) return fail(AGS_E_ARG, "bind: bad arguments");
  S->bound[which] = ptr;
  return AGS_OK;
}

extern "C" int ags_sim_step(ags_sim* S, void* stream) {
  if (!S) return fail(AGS_E_ARG, "step: null sim");
  if (!S->bound[AGS_ROOT_STATE] || !S->bound[AGS_DOF_STATE] || !S->bound[AGS_DOF_ACTUATION])
    return fail(AGS_E_UNBOUND, "step: root state, DOF state and DOF actuation tensors must be bound");
  const ags_sim_params& p = S->params;
  const bool rows_dbg = S->bound[AGS_DEBUG_ROW_COUNT] && S->bound[AGS_DEBUG_ROW_KEY] && S->bound[AGS_DEBUG_ROW_LAMBDA];
  StepArgs a{};
  a.env_actor_base = S->env_tables;
  a.env_dof_base = S->env_tables + S->n_envs;
  a.env_body_base = S->env_tables + 2 * S->n_envs;
  a.root_state = (float*)S->bound[AGS_ROOT_STATE];
  a.dof_state = (float*)S->bound[AGS_DOF_STATE];
  a.act = (const float*)S->bound[AGS_DOF_ACTUATION];
  a.pos_tgt = (const float*)S->bound[AGS_DOF_POS_TARGET];
  a.vel_tgt = (const float*)S->bound[AGS_DOF_VEL_TARGET];
  a.contact_force = (float*)S->bound[AGS_NET_CONTACT_FORCE];
  a.rb_state = (float*)S->bound[AGS_RIGID_BODY_STATE];
  a.env_status = (int*)S->bound[AGS_ENV_STATUS];
  a.big_rows = S->big_out;
  a.mass_scale = (const float*)S->bound[AGS_BODY_MASS_SCALE];
  a.dof_kp = (const float*)S->bound[AGS_DOF_STIFFNESS];
  a.dof_kd = (const float*)S->bound[AGS_DOF_DAMPING];
  a.dof_limits = (const float*)S->bound[AGS_DOF_LIMITS];
  a.env_mu = (const float*)S->bound[AGS_ENV_FRICTION];
  a.env_gravity = (const float*)S->bound[AGS_ENV_GRAVITY];
  a.dof_force = (float*)S->bound[AGS_DOF_FORCE];
  a.dbg_qdd = (float*)S->bound[AGS_DEBUG_QDD_FREE];
  a.dbg_qdd_stride = p.substeps * S->max_nv;
  a.dbg_qdd_sub = S->max_nv;
  a.dbg_rc = rows_dbg ? (int*)S->bound[AGS_DEBUG_ROW_COUNT] : nullptr;
  a.dbg_key = rows_dbg ? (int*)S->bound[AGS_DEBUG_ROW_KEY] : nullptr;
  a.dbg_lam = rows_dbg ? (float*)S->bound[AGS_DEBUG_ROW_LAMBDA] : nullptr;
  a.dbg_row_stride = p.substeps * std::max(1, S->max_rows);
  a.dbg_row_sub = std::max(1, S->max_rows);
  a.dbg_cycles = (long long*)S->bound[AGS_DEBUG_PHASE_CYCLES];
  a.mid_root = S->mid_root;
  a.mid_dof = S->mid_root ? S->mid_root + 13ll * S->n_actors_total : nullptr;
  a.mid_block = 13ll * S->n_actors_total + 2ll * S->n_dof_total;
  a.dt = p.dt;
  a.h = (double)p.dt / p.substeps;
  a.gx = p.gravity[0];
  a.gy = p.gravity[1];
  a.gz = p.gravity[2];
  a.mu = p.mu;
  a.beta = p.baumgarte;
  a.mc = p.contact_margin;
  a.substeps = p.substeps;
  a.iters = p.pgs_iters;
  a.solver = p.solver;
  auto type_args = [](const TypeDev& T) {
    TypeArgs t{};
    t.m = T.dm;
    t.lds = T.lds;
    t.env_list = T.env_list;
    t.n_envs = T.n_envs;
    t.scratch = T.scratch;
    t.scratch_stride = T.scratch_stride;
    return t;
  };
  if (S->fused_ok) {
    FusedArgs f{};
    f.base = a;
    for (size_t k = 0; k < S->types.size(); ++k) f.types[k] = type_args(S->types[k]);
    f.units = S->units;
    f.n_units = S->n_units;
    hipError_t e = launch_step_fused(f, S->fused_grid, S->fused_lds, p.compute_fp64, S->fused_team, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "step: launch");
    return AGS_OK;
  }
  // A launch ends with its slowest workgroups, and an env-step's cost grows with its constraint rows (those
  // past 32 take the chunked response path): one-env-per-wavefront types dispatch their envs in order of
  // the rows of their previous step, most first, so that the likely slow ones start in the first round of
  // workgroups.  The order changes no result: every env is computed on its own.
  a.env_rows = S->env_rows;
  for (TypeDev& T : S->types) {
    a.ty = type_args(T);
    if (T.step_order) a.ty.env_list = T.step_order;
    hipError_t e = launch_step(a, T.n_envs, p.compute_fp64, T.team, (hipStream_t)stream);
    if (e == hipSuccess && T.step_order)
      e = launch_order_by_rows(T.step_order, T.order_tmp, S->env_rows, T.n_envs, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "step: launch");
  }
  return AGS_OK;
}

namespace {
// what the adjoint does not differentiate, or NULL
const char* adjoint_unsupported(const ags_sim* S) {
  if (S->params.solver != AGS_SOLVER_PGS) return "adjoint: supports the projected Gauss-Seidel solver only";
  for (const TypeDev& T : S->types)
    if (T.dm.n_tj > 0) return "adjoint: models with tendons are not supported";
  for (int w = AGS_BODY_MASS_SCALE; w <= AGS_ENV_GRAVITY; ++w)
    if (S->bound[w]) return "adjoint: per-env property tensors are not supported";
  return nullptr;
}
}  // namespace

extern "C" int ags_sim_step_backward(ags_sim* S, const float* root_state, const float* dof_state,
                                     const float* actuation, float* root_adj, float* dof_adj, float* act_adj,
                                     int32_t* status, void* stream) {
  if (!S || !root_state || !dof_state || !actuation || !root_adj || !dof_adj || !act_adj)
    return fail(AGS_E_ARG, "step_backward: bad arguments");
  const ags_sim_params& p = S->params;
  if (p.pgs_iters > kAdjIters) return fail(AGS_E_ARG, "step_backward: more Gauss-Seidel sweeps than the adjoint's tape holds (32)");
  if (const char* why = adjoint_unsupported(S)) return fail(AGS_E_ARG, why);
  for (const TypeDev& T : S->types) {
    if (T.adj_bytes > 160 * 1024) return fail(AGS_E_ARG, "step_backward: model too large for one workgroup's LDS");
  }
  for (TypeDev& T : S->types) {
    AdjArgs a{};
    a.m = T.dm;
    a.L = T.adj;
    a.env_list = T.env_list;
    a.env_actor_base = S->env_tables;
    a.env_dof_base = S->env_tables + S->n_envs;
    a.root_state = root_state;
    a.dof_state = dof_state;
    a.act = actuation;
    a.pos_tgt = (const float*)S->bound[AGS_DOF_POS_TARGET];
    a.vel_tgt = (const float*)S->bound[AGS_DOF_VEL_TARGET];
    a.root_adj = root_adj;
    a.dof_adj = dof_adj;
    a.act_adj = act_adj;
    a.status = status;
    a.status_sticky = S->adj_sticky;
    a.cycles = (long long*)S->bound[AGS_DEBUG_ADJ_CYCLES];
    a.mid_root = S->mid_root;
    a.mid_dof = S->mid_root ? S->mid_root + 13ll * S->n_actors_total : nullptr;
    a.mid_block = 13ll * S->n_actors_total + 2ll * S->n_dof_total;
    a.h = (double)p.dt / p.substeps;
    a.gx = p.gravity[0];
    a.gy = p.gravity[1];
    a.gz = p.gravity[2];
    a.mu = p.mu;
    a.beta = p.baumgarte;
    a.mc = p.contact_margin;
    a.substeps = p.substeps;
    a.iters = p.pgs_iters;
    hipError_t e = hipSuccess;
    if (T.adj_two) {
      // pass 1 with the small layout (more workgroups per CU); environments with more rows are collected
      // and pass 2 runs them with the full layout
      AdjArgs a1 = a;
      a1.L = T.adj_small;
      a1.retry_count = S->adj_retry;
      a1.retry = S->adj_retry + 1;
      AdjArgs a2 = a;
      a2.env_list = S->adj_retry + 1;
      a2.list_count = S->adj_retry;
      const hipStream_t st = (hipStream_t)stream;
      if (S->adj_big) {
        // environments the forward flagged run with the full layout on the third stream, concurrently with
        // pass 1 (which skips them): a device list of them, strided over by a few workgroups per CU (a launch
        // of one workgroup per env would wait for LDS room for each of its mostly empty workgroups); the
        // caller's stream waits for them before its next work.  A batch of at most 16 envs per CU has about
        // as many flagged envs as CUs: one workgroup per CU, and pass 1 released only once the flagged list
        // is built, when the flagged launch is already queued behind it on the third stream, so that its
        // workgroups find LDS room before pass 1's fill the CUs (started together, they waited for pass 1's
        // workgroups to finish and ended last).  64-step reverse pass of 4096 humanoids: FP64 adjoint 236 ->
        // 213 ms, FP32 adjoint 127.0 ms (two per CU, started together) -> 124.1 ms.  Larger batches have many
        // flagged envs and the launch is bound by throughput: as many workgroups per CU as LDS holds beside one
        // of pass 1 (at most two), started together with pass 1 unless that is one (32-step reverse pass of
        // 65536 hand-like envs, FP32 adjoint: 1144 ms, against 1236 ms with one per CU queued first).
        const int fit =
            std::max(1, std::min(2, (int)((160 * 1024 - (long long)T.adj_small_bytes) / (long long)T.adj_bytes)));
        const int big_per_cu = T.n_envs <= 16 * S->n_cu ? 1 : fit;
        const bool gate = big_per_cu == 1;
        a1.skip_flags = S->adj_big;
        AdjArgs ab = a;
        ab.env_list = S->adj_big_list + 1;
        ab.list_count = S->adj_big_list;
        if ((e = hipEventRecord(S->ev_big_start, st)) == hipSuccess &&
            (e = hipStreamWaitEvent(S->aux2, S->ev_big_start, 0)) == hipSuccess &&
            (e = launch_zero_count(S->adj_big_list, S->aux2)) == hipSuccess &&
            (e = launch_compact_flags(T.env_list, T.n_envs, S->adj_big, S->adj_big_list, S->aux2)) == hipSuccess &&
            (e = hipEventRecord(S->ev_big_listed, S->aux2)) == hipSuccess &&
            (e = launch_adjoint(ab, T.n_envs, adj_fp64(p), S->aux2, S->n_cu * big_per_cu)) == hipSuccess)
          e = hipEventRecord(S->ev_big_done, S->aux2);
        if (e == hipSuccess && gate) e = hipStreamWaitEvent(st, S->ev_big_listed, 0);
        if (e != hipSuccess) return hip_fail(e, "step_backward: flagged pass");
      }
      if ((e = launch_zero_count(S->adj_retry, st)) == hipSuccess &&
          (e = launch_adjoint(a1, T.n_envs, adj_fp64(p), st)) == hipSuccess)
        e = launch_adjoint(a2, T.n_envs, adj_fp64(p), st);
      if (e == hipSuccess && S->adj_big) e = hipStreamWaitEvent(st, S->ev_big_done, 0);
    } else {
      e = launch_adjoint(a, T.n_envs, adj_fp64(p), (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "step_backward: launch");
  }
  return AGS_OK;
}

// ---------------------------------------------------------------- Jacobian and mass-matrix tensors
extern "C" int ags_sim_jacobian_mass(ags_sim* S, int32_t model, float* jac, float* mass, void* stream) {
  if (!S || (!jac && !mass)) return fail(AGS_E_ARG, "jacobian_mass: bad arguments");
  if (!S->bound[AGS_ROOT_STATE] || !S->bound[AGS_DOF_STATE])
    return fail(AGS_E_UNBOUND, "jacobian_mass: root and DOF state tensors must be bound");
  const TypeDev* T = nullptr;
  for (const TypeDev& t : S->types)
    if (t.model == model) T = &t;
  if (!T) return fail(AGS_E_ARG, "jacobian_mass: no environment uses this model");
  if (jacmass_lds_bytes(T->dm.n_links, T->dm.n_v) > 64 * 1024) return fail(AGS_E_ARG, "jacobian_mass: model too large");
  JacMassArgs a{};
  a.m = T->dm;
  a.env_list = T->env_list;
  a.n_envs = T->n_envs;
  a.env_actor_base = S->env_tables;
  a.env_dof_base = S->env_tables + S->n_envs;
  a.root_state = (const float*)S->bound[AGS_ROOT_STATE];
  a.dof_state = (const float*)S->bound[AGS_DOF_STATE];
  a.jac = jac;
  a.mass = mass;
  a.env_body_base = S->env_tables + 2 * S->n_envs;
  a.mass_scale = (const float*)S->bound[AGS_BODY_MASS_SCALE];
  const hipError_t e = launch_jacmass(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "jacobian_mass: launch");
  return AGS_OK;
}

// ---------------------------------------------------------------- rollouts with checkpoints
extern "C" int ags_rollout_state_size(const ags_sim* S, int64_t* floats) {
  if (!S || !floats) return fail(AGS_E_ARG, "rollout_state_size: bad arguments");
  *floats = 13ll * S->n_actors_total + 2ll * S->n_dof_total;
  return AGS_OK;
}

namespace {
long long seg_one_bytes(const ags_sim* S, int every);
}

extern "C" int ags_rollout_seg_bytes(const ags_sim* S, int32_t every, int64_t* bytes) {
  if (!S || every < 1 || !bytes) return fail(AGS_E_ARG, "rollout_seg_bytes: bad arguments");
  *bytes = 2 * seg_one_bytes(S, every);  // two segment buffers (recompute of one overlaps the adjoint of the other)
  return AGS_OK;
}

namespace {
// one env-step on the given state arrays with the given control; the output tensors are not written
// bytes of one segment buffer: every + 1 FP32 states (256-byte aligned), then every x (substeps - 1) FP64
// states, then every x n_envs row-count flags
long long seg_one_bytes(const ags_sim* S, int every) {
  const long long sw = 13ll * S->n_actors_total + 2ll * S->n_dof_total;
  const long long mid = (long long)every * std::max(0, S->params.substeps - 1) * sw;
  const long long flags = ((long long)every * S->n_envs * (long long)sizeof(int) + 255) / 256 * 256;
  return (((every + 1) * sw * (long long)sizeof(float) + 255) / 256 * 256 + mid * (long long)sizeof(double) + 255) / 256 * 256 +
         flags;
}

int step_on(ags_sim* S, float* root, float* dof, int control, const float* ctrl, hipStream_t stream) {
  void* saved[AGS_NUM_TENSORS];
  std::memcpy(saved, S->bound, sizeof(saved));
  for (int w = AGS_NET_CONTACT_FORCE; w <= AGS_ENV_STATUS; ++w) S->bound[w] = nullptr;  // outputs only
  S->bound[AGS_ROOT_STATE] = root;
  S->bound[AGS_DOF_STATE] = dof;
  S->bound[control] = const_cast<float*>(ctrl);
  const int rc = ags_sim_step(S, stream);
  std::memcpy(S->bound, saved, sizeof(saved));
  return rc;
}

// the adjoints of steps t1-1 down to t0 of a segment: x holds the FP32 state before each of its steps,
// mid the FP64 substep states and flags the row-count flags of each step (both from the step's forward)
int reverse_steps(ags_sim* S, int t0, int t1, int control, const float* actions, const float* x, const double* mid,
                  const int* flags, float* root_adj, float* dof_adj, float* act_adj, int32_t* status, hipStream_t st) {
  const size_t nr = 13ull * S->n_actors_total, sw = nr + 2ull * S->n_dof_total;
  const size_t na = (size_t)S->n_dof_total;
  const int nmid = std::max(0, S->params.substeps - 1);
  S->adj_sticky = 1;
  struct Unsticky {
    ags_sim* s;
    ~Unsticky() { s->adj_sticky = 0; }
  } unsticky{S};
  for (int t = t1 - 1; t >= t0; --t) {
    const float* xt = x + (size_t)(t - t0) * sw;
    void* saved = S->bound[control];
    S->bound[control] = const_cast<float*>(actions + (size_t)t * na);
    // the actuation the step used: the per-step array or the bound tensor
    const float* act = (const float*)S->bound[AGS_DOF_ACTUATION];
    S->mid_root = nmid ? const_cast<double*>(mid) + (size_t)(t - t0) * nmid * sw : nullptr;
    S->adj_big = flags + (size_t)(t - t0) * S->n_envs;
    int rc = ags_sim_step_backward(S, xt, xt + nr, act, root_adj, dof_adj, act_adj + (size_t)t * na, status, st);
    S->mid_root = nullptr;
    S->adj_big = nullptr;
    S->bound[control] = saved;
    if (rc == AGS_OK && control == AGS_DOF_POS_TARGET) {
      // the target enters the step only through tau = ... + kp q*: dL/dq* = kp dL/dtau
      const hipError_t e2 = launch_scale_by_kp(act_adj + (size_t)t * na, S->kp_dof, (int)na, st);
      if (e2 != hipSuccess) rc = hip_fail(e2, "rollout_backward: target adjoint");
    }
    if (rc != AGS_OK) return rc;
  }
  return AGS_OK;
}

// the rollout's extra streams and events, created on first use on the sim's current device; default priority
hipError_t ensure_streams(ags_sim* S) {
  if (S->aux) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&S->aux, hipStreamNonBlocking);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&S->ev_ready[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_free[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->aux2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_big_start, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_big_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_big_listed, hipEventDisableTiming);
  return e;
}

// where the parts of a segment buffer of `every` steps start (the layout of seg_one_bytes)
void seg_parts(const ags_sim* S, void* base, int every, float** x, double** mid, int** flags) {
  const size_t sw = 13ull * S->n_actors_total + 2ull * S->n_dof_total;
  const size_t nmid = (size_t)std::max(0, S->params.substeps - 1);
  const size_t states_bytes = ((every + 1) * sw * sizeof(float) + 255) / 256 * 256;
  const size_t mid_bytes = ((size_t)every * nmid * sw * sizeof(double) + 255) / 256 * 256;
  char* b = static_cast<char*>(base);
  *x = reinterpret_cast<float*>(b);
  *mid = reinterpret_cast<double*>(b + states_bytes);
  *flags = reinterpret_cast<int*>(b + states_bytes + mid_bytes);
}
}  // namespace

extern "C" int ags_rollout_forward(ags_sim* S, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                                   float* ckpt, void* stream) {
  if (!S || n_steps < 1 || every < 1 || !actions || !ckpt || (control != AGS_DOF_ACTUATION && control != AGS_DOF_POS_TARGET))
    return fail(AGS_E_ARG, "rollout_forward: bad arguments");
  if (!S->bound[AGS_DOF_ACTUATION]) return fail(AGS_E_UNBOUND, "rollout_forward: the actuation tensor must be bound");
  if (!S->bound[AGS_ROOT_STATE] || !S->bound[AGS_DOF_STATE])
    return fail(AGS_E_UNBOUND, "rollout_forward: root and DOF state tensors must be bound");
  const size_t nr = 13ull * S->n_actors_total, nd = 2ull * S->n_dof_total, sw = nr + nd;
  hipStream_t st = (hipStream_t)stream;
  float* root = (float*)S->bound[AGS_ROOT_STATE];
  float* dof = (float*)S->bound[AGS_DOF_STATE];
  for (int t = 0; t < n_steps; ++t) {
    if (t % every == 0) {
      float* c = ckpt + (size_t)(t / every) * sw;
      hipError_t e = hipMemcpyAsync(c, root, nr * sizeof(float), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(c + nr, dof, nd * sizeof(float), hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "rollout_forward: checkpoint copy");
    }
    void* saved = S->bound[control];
    S->bound[control] = const_cast<float*>(actions + (size_t)t * S->n_dof_total);
    const int rc = ags_sim_step(S, stream);
    S->bound[control] = saved;
    if (rc != AGS_OK) return rc;
  }
  return AGS_OK;
}

namespace {
int rollout_backward(ags_sim* S, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                     const float* ckpt, void* seg_bytes, float* root_adj, float* dof_adj, float* act_adj,
                     int32_t* status, void* stream);
}

extern "C" int ags_rollout_backward(ags_sim* S, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                                    const float* ckpt, void* seg_bytes, float* root_adj, float* dof_adj, float* act_adj,
                                    int32_t* status, void* stream) {
  if (!S || n_steps < 1 || every < 1 || !actions || !ckpt || !seg_bytes || !root_adj || !dof_adj || !act_adj ||
      (control != AGS_DOF_ACTUATION && control != AGS_DOF_POS_TARGET))
    return fail(AGS_E_ARG, "rollout_backward: bad arguments");
  return rollout_backward(S, n_steps, every, control, actions, ckpt, seg_bytes, root_adj, dof_adj, act_adj, status,
                          stream);
}

extern "C" int ags_rollout_backward_noalloc(ags_sim* S, int32_t n_steps, int32_t every, int32_t control,
                                            const float* actions, const float* ckpt, float* root_adj, float* dof_adj,
                                            float* act_adj, int32_t* status, void* stream) {
  if (!S || n_steps < 1 || every < 1 || !actions || !ckpt || !root_adj || !dof_adj || !act_adj ||
      (control != AGS_DOF_ACTUATION && control != AGS_DOF_POS_TARGET))
    return fail(AGS_E_ARG, "rollout_backward_noalloc: bad arguments");
  if (!S->noalloc_scratch) return fail(AGS_E_ARG, "rollout_backward_noalloc: no scratch on this sim's device");
  const long long need = 2 * seg_one_bytes(S, every);
  if (need > kNoAllocScratchBytes)
    return fail(AGS_E_ARG, "rollout_backward_noalloc: two segment buffers of this sim and checkpoint interval need " +
                               std::to_string(need) + " bytes, more than the " + std::to_string(kNoAllocScratchBytes) +
                               " bytes of the static scratch; use a smaller interval or ags_rollout_backward");
  return rollout_backward(S, n_steps, every, control, actions, ckpt, S->noalloc_scratch, root_adj, dof_adj, act_adj,
                          status, stream);
}

namespace {
// the reverse pass of a checkpointed rollout with its two segment buffers at seg_bytes (arguments checked)
int rollout_backward(ags_sim* S, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                     const float* ckpt, void* seg_bytes, float* root_adj, float* dof_adj, float* act_adj,
                     int32_t* status, void* stream) {
  if (!S->bound[AGS_DOF_ACTUATION]) return fail(AGS_E_UNBOUND, "rollout_backward: the actuation tensor must be bound");
  if (const char* why = adjoint_unsupported(S)) return fail(AGS_E_ARG, why);
  const size_t nr = 13ull * S->n_actors_total, nd = 2ull * S->n_dof_total, sw = nr + nd;
  const size_t na = (size_t)S->n_dof_total;
  const int nmid = std::max(0, S->params.substeps - 1);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if ((e = ensure_streams(S)) != hipSuccess) return hip_fail(e, "rollout_backward: streams");
  // two segment buffers, each: every + 1 FP32 states, then every x nmid FP64 substep states, then every x
  // n_envs flags
  const long long one = seg_one_bytes(S, every);
  float* seg[2];
  double* mid[2];
  int* flags[2];
  for (int k = 0; k < 2; ++k) seg_parts(S, static_cast<char*>(seg_bytes) + k * one, every, &seg[k], &mid[k], &flags[k]);
  const int n_seg = (n_steps + every - 1) / every;
  // recompute segment g into buffer g % 2 on the auxiliary stream: the states before its steps (the last
  // step's end state is discarded) and the substep states of every step
  auto recompute = [&](int g) -> int {
    const int b = g & 1, t0 = g * every, t1 = std::min(n_steps, t0 + every);
    hipError_t e2;
    if ((e2 = hipStreamWaitEvent(S->aux, S->ev_free[b], 0)) != hipSuccess) return hip_fail(e2, "rollout_backward: wait");
    if ((e2 = hipMemcpyAsync(seg[b], ckpt + (size_t)g * sw, sw * sizeof(float), hipMemcpyDeviceToDevice, S->aux)) != hipSuccess)
      return hip_fail(e2, "rollout_backward: copy");
    for (int t = t0; t < t1; ++t) {
      float* a = seg[b] + (size_t)(t - t0) * sw;
      float* x = a + sw;
      if ((e2 = hipMemcpyAsync(x, a, sw * sizeof(float), hipMemcpyDeviceToDevice, S->aux)) != hipSuccess)
        return hip_fail(e2, "rollout_backward: copy");
      S->mid_root = nmid ? mid[b] + (size_t)(t - t0) * nmid * sw : nullptr;
      S->big_out = flags[b] + (size_t)(t - t0) * S->n_envs;
      const int rc = step_on(S, x, x + nr, control, actions + (size_t)t * na, S->aux);
      S->mid_root = nullptr;
      S->big_out = nullptr;
      if (rc != AGS_OK) return rc;
    }
    if ((e2 = hipEventRecord(S->ev_ready[b], S->aux)) != hipSuccess) return hip_fail(e2, "rollout_backward: record");
    return AGS_OK;
  };
  // both buffers start free once the caller's earlier work on the stream is done
  for (int k = 0; k < 2; ++k)
    if ((e = hipEventRecord(S->ev_free[k], st)) != hipSuccess) return hip_fail(e, "rollout_backward: record");
  if (status && (e = launch_fill_int(status, S->n_envs, 0, st)) != hipSuccess)
    return hip_fail(e, "rollout_backward: clear status");
  int rc = recompute(n_seg - 1);
  if (rc != AGS_OK) return rc;
  for (int g = n_seg - 1; g >= 0; --g) {
    const int b = g & 1, t0 = g * every, t1 = std::min(n_steps, t0 + every);
    if (g > 0 && (rc = recompute(g - 1)) != AGS_OK) return rc;  // overlaps the adjoints below
    if ((e = hipStreamWaitEvent(st, S->ev_ready[b], 0)) != hipSuccess) return hip_fail(e, "rollout_backward: wait");
    if ((rc = reverse_steps(S, t0, t1, control, actions, seg[b], mid[b], flags[b], root_adj, dof_adj, act_adj, status,
                            st)) != AGS_OK)
      return rc;
    if ((e = hipEventRecord(S->ev_free[b], st)) != hipSuccess) return hip_fail(e, "rollout_backward: record");
  }
  return AGS_OK;
}
}  // namespace

// ---------------------------------------------------------------- rollouts with a stored tape
extern "C" int ags_rollout_tape_bytes(const ags_sim* S, int32_t n_steps, int64_t* bytes) {
  if (!S || n_steps < 1 || !bytes) return fail(AGS_E_ARG, "rollout_tape_bytes: bad arguments");
  *bytes = seg_one_bytes(S, n_steps);
  return AGS_OK;
}

extern "C" int ags_rollout_forward_tape(ags_sim* S, int32_t n_steps, int32_t control, const float* actions, void* tape,
                                        void* stream) {
  if (!S || n_steps < 1 || !actions || !tape || (control != AGS_DOF_ACTUATION && control != AGS_DOF_POS_TARGET))
    return fail(AGS_E_ARG, "rollout_forward_tape: bad arguments");
  if (!S->bound[AGS_DOF_ACTUATION]) return fail(AGS_E_UNBOUND, "rollout_forward_tape: the actuation tensor must be bound");
  if (!S->bound[AGS_ROOT_STATE] || !S->bound[AGS_DOF_STATE])
    return fail(AGS_E_UNBOUND, "rollout_forward_tape: root and DOF state tensors must be bound");
  const size_t nr = 13ull * S->n_actors_total, nd = 2ull * S->n_dof_total, sw = nr + nd;
  const int nmid = std::max(0, S->params.substeps - 1);
  hipStream_t st = (hipStream_t)stream;
  float* x;
  double* mid;
  int* flags;
  seg_parts(S, tape, n_steps, &x, &mid, &flags);
  float* root = (float*)S->bound[AGS_ROOT_STATE];
  float* dof = (float*)S->bound[AGS_DOF_STATE];
  for (int t = 0; t < n_steps; ++t) {
    float* c = x + (size_t)t * sw;
    hipError_t e = hipMemcpyAsync(c, root, nr * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c + nr, dof, nd * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "rollout_forward_tape: state copy");
    void* saved = S->bound[control];
    S->bound[control] = const_cast<float*>(actions + (size_t)t * S->n_dof_total);
    S->mid_root = nmid ? mid + (size_t)t * nmid * sw : nullptr;
    S->big_out = flags + (size_t)t * S->n_envs;
    const int rc = ags_sim_step(S, stream);
    S->mid_root = nullptr;
    S->big_out = nullptr;
    S->bound[control] = saved;
    if (rc != AGS_OK) return rc;
  }
  return AGS_OK;
}

extern "C" int ags_rollout_backward_tape(ags_sim* S, int32_t n_steps, int32_t control, const float* actions,
                                         const void* tape, float* root_adj, float* dof_adj, float* act_adj,
                                         int32_t* status, void* stream) {
  if (!S || n_steps < 1 || !actions || !tape || !root_adj || !dof_adj || !act_adj ||
      (control != AGS_DOF_ACTUATION && control != AGS_DOF_POS_TARGET))
    return fail(AGS_E_ARG, "rollout_backward_tape: bad arguments");
  if (!S->bound[AGS_DOF_ACTUATION]) return fail(AGS_E_UNBOUND, "rollout_backward_tape: the actuation tensor must be bound");
  if (const char* why = adjoint_unsupported(S)) return fail(AGS_E_ARG, why);
  hipError_t e = ensure_streams(S);
  if (e != hipSuccess) return hip_fail(e, "rollout_backward_tape: streams");
  float* x;
  double* mid;
  int* flags;
  seg_parts(S, const_cast<void*>(tape), n_steps, &x, &mid, &flags);
  if (status && (e = launch_fill_int(status, S->n_envs, 0, (hipStream_t)stream)) != hipSuccess)
    return hip_fail(e, "rollout_backward_tape: clear status");
  return reverse_steps(S, 0, n_steps, control, actions, x, mid, flags, root_adj, dof_adj, act_adj, status,
                       (hipStream_t)stream);
}

// ---------------------------------------------------------------- autotuner
extern "C" int ags_autotune(const ags_model* const* models, int32_t n_models, const int32_t* env_model, int32_t n_envs,
                            ags_sim_params* params, const float* root_state, const float* dof_state,
                            const float* actuation, int32_t n_steps, float* ms_out, void* stream) {
  if (!models || !env_model || !params || !root_state || !dof_state || !actuation || n_steps < 1)
    return fail(AGS_E_ARG, "autotune: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  // candidate mappings: lanes per environment x persistent launch
  std::vector<std::pair<int, int>> cands;
  bool small = true;
  for (int e = 0; e < n_envs; ++e)
    if (env_model[e] < 0 || env_model[e] >= n_models || !models[env_model[e]]) return fail(AGS_E_ARG, "autotune: bad env model index");
    else if (models[env_model[e]]->info.n_v > 32) small = false;
  for (int lanes : {64, 32}) {
    if (lanes == 32 && !small) continue;
    for (int per : {0, 1}) cands.push_back({lanes, per});
  }
  ags_sim* probe = nullptr;
  ags_sim_params p0 = *params;
  p0.lanes_per_env = 64;
  p0.persistent = 0;
  int rc = ags_sim_create(models, n_models, env_model, n_envs, &p0, &probe);
  if (rc != AGS_OK) return rc;
  const size_t nr = 13ull * probe->n_actors_total, nd = 2ull * probe->n_dof_total, na = probe->n_dof_total;
  ags_sim_destroy(probe);
  float *root = nullptr, *dof = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&root, nr * sizeof(float))) != hipSuccess) return hip_fail(e, "autotune: state copy");
  if ((e = hipMalloc(&dof, nd * sizeof(float))) != hipSuccess) {
    (void)hipFree(root);
    return hip_fail(e, "autotune: state copy");
  }
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  float best = 1e30f;
  std::pair<int, int> pick = cands[0];
  int status = AGS_OK;
  for (auto c : cands) {
    ags_sim_params pc = *params;
    pc.lanes_per_env = c.first;
    pc.persistent = c.second;
    ags_sim* S = nullptr;
    if (ags_sim_create(models, n_models, env_model, n_envs, &pc, &S) != AGS_OK) continue;  // mapping not possible
    S->bound[AGS_ROOT_STATE] = root;
    S->bound[AGS_DOF_STATE] = dof;
    S->bound[AGS_DOF_ACTUATION] = const_cast<float*>(actuation);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && status == AGS_OK; ++rep) {  // the first repetition warms up
      if ((e = hipMemcpyAsync(root, root_state, nr * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
          (e = hipMemcpyAsync(dof, dof_state, nd * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
          (e = hipEventRecord(a, st)) != hipSuccess) {
        status = hip_fail(e, "autotune: copy");
        break;
      }
      for (int t = 0; t < n_steps && status == AGS_OK; ++t) status = ags_sim_step(S, stream);
      if (status == AGS_OK && ((e = hipEventRecord(b, st)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
                               (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess))
        status = hip_fail(e, "autotune: timing");
    }
    ags_sim_destroy(S);
    if (status != AGS_OK) break;
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(root);
  (void)hipFree(dof);
  (void)na;
  if (status != AGS_OK) return status;
  params->lanes_per_env = pick.first;
  params->persistent = pick.second;
  if (ms_out) *ms_out = best / n_steps;
  return AGS_OK;
}

static int set_indexed(ags_sim* S, int which, const float* src, const int32_t* idx, int32_t n, void* stream) {
  if (!S || !src || n < 0 || (!idx && n != 0 && n != S->n_actors_total)) return fail(AGS_E_ARG, "set: bad arguments");
  if (!S->bound[which]) return fail(AGS_E_UNBOUND, "set: target tensor not bound");
  if (n == 0) return AGS_OK;  // an empty list sets nothing (its pointer may be NULL)
  const int width = which == AGS_ROOT_STATE ? 13 : 2;
  hipError_t e = launch_set_rows((float*)S->bound[which], src, idx, idx ? n : S->n_actors_total, S->n_actors_total,
                                 S->actor_rows, which == AGS_ROOT_STATE ? 0 : 2, width, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "set: launch");
  return AGS_OK;
}

extern "C" int ags_sim_set_root_state_indexed(ags_sim* S, const float* src, const int32_t* idx, int32_t n,
                                              void* stream) {
  return set_indexed(S, AGS_ROOT_STATE, src, idx, n, stream);
}

extern "C" int ags_sim_set_dof_state_indexed(ags_sim* S, const float* src, const int32_t* idx, int32_t n,
                                             void* stream) {
  return set_indexed(S, AGS_DOF_STATE, src, idx, n, stream);
}
