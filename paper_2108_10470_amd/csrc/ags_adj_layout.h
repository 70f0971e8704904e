// LDS layout of the adjoint kernel (one environment per 64-lane workgroup): plain C++ with no HIP
// dependency, shared by the host runtime and the host-side layout checker of the tests.
#pragma once

#include <algorithm>

#include "../../include/ags.h"

namespace ags {

constexpr int kAdjRows = 64;   // constraint rows per substep the adjoint handles (one lane each)
constexpr int kAdjSmallRows = 32;  // row capacity of the first, smaller-LDS adjoint pass
constexpr int kAdjBigRowsAt = 29;  // rows above which the forward flags an env for the larger layout (one contact's margin)
constexpr int kAdjIters = 32;  // Gauss-Seidel sweeps the adjoint's tape holds
constexpr int kAdjPhases = 11;  // see AGS_DEBUG_ADJ_CYCLES
constexpr int kLinkIntCols = 10;  // ints per link of the model's link table

// per-environment LDS layout of the adjoint kernel: offsets in elements of the compute type (reals)
// or in ints (integer region, placed after the reals)
struct AdjLds {
  int Rm, p, ax, c, Iw, Ic, V, Vs, X0, X1, X2, X3, wr, sb, cb, tI;  // per link (X0, X2, X3 in A's words; wr..tI in the tape's)
  int nu, qdd, vs, nu1, tau, arm, z, w, nub, vsb, nui, tmp;        // per column
  int colS, colY, colYv, cs;                                       // per column, 6 each
  int q, qb, ab;                                                   // per DOF
  int st, rbar, dbar, nrb;                                             // state of each substep start, state adjoint
  int Lm, nvp, ldi;  // packed lower triangle of an n_v x n_v matrix (factor, then P); row stride of J, W; 1 / diag of the factor
  int J, W, A, Ab, rcp;  // rows: J, W (rows x nvp); A and S = Abar + Abar^T (packed symmetric)
  int rbc, rb, rinvA, rlam, rybar, rbbar, rx, rcen, rd, rxb, rqb;  // per row reals
  int rdb, rwa, rwb;                                               // per row: d adjoint, wrenches of bodies a, b
  int hlo, hres;                                                   // tape: iters x rcp
  int misc;
  int n_real;
  // integer region
  int rkind, rlink, rdof, rnrm, rmap, rlinkb, rslot, hst, flags;
  // the model's integer tables staged once per workgroup: link table, level starts (at most one level per
  // link, plus the end), links by level, children, link of each column, link of each DOF
  int t_li, t_lev, t_links, t_child, t_col, t_dof;
  int n_int;
  int state_words;  // reals of one stored state: 13 per actor + 2 per DOF
  int rows_cap;     // min(max rows, kAdjRows)
};

// LDS layout of the adjoint kernel for one environment (one wavefront per environment)
// stage_tables: room for the model's integer tables in the integer region (the FP64 forms, whose LDS holds two
// workgroups per CU with room to spare; the FP32 forms keep reading them through the caches, since the
// tables would cost their small layout a workgroup per CU)
inline AdjLds make_adj_layout(const ags_model_info& info, int substeps, int iters, int row_cap, bool stage_tables) {
  AdjLds L{};
  int off = 0;
  auto take = [&](int n) {
    const int o = off;
    off += std::max(n, 1);
    return o;
  };
  const int nl = info.n_links, nv = std::max(1, info.n_v), nd = std::max(1, info.n_dof), na = info.n_actors;
  const int rc = std::min(std::max(1, info.max_rows), row_cap);
  L.rows_cap = rc;
  L.Rm = take(9 * nl); L.p = take(3 * nl); L.ax = take(3 * nl); L.c = take(3 * nl); L.Iw = take(6 * nl);
  L.Ic = take(10 * nl); L.V = take(6 * nl); L.Vs = take(6 * nl); L.X1 = take(6 * nl);
  L.nu = take(nv); L.qdd = take(nv); L.vs = take(nv); L.nu1 = take(nv); L.tau = take(nv); L.arm = take(nv);
  L.z = take(nv); L.w = take(nv); L.nub = take(nv); L.vsb = take(nv); L.nui = take(nv); L.tmp = take(nv);
  L.cs = take(6 * nv);
  L.q = take(nd); L.qb = take(nd); L.ab = take(nd);
  L.state_words = 13 * na + 2 * info.n_dof;
  L.st = take((substeps + 1) * L.state_words);
  L.rbar = take(13 * na); L.dbar = take(2 * nd); L.nrb = take(13 * na);
  L.nvp = nv | 1;
  L.Lm = take(nv * (nv + 1) / 2);  // entry (i, j), j <= i, at i (i + 1) / 2 + j
  L.ldi = take(nv);
  L.rcp = rc | 1;
  // arrays with disjoint lifetimes share words: W is dead once P is formed, when the mass-matrix terms' column
  // vectors are written; A and S = Abar + Abar^T are dead after the reverse Gauss-Seidel and T = S W, when
  // the reverse RNEA's per-link temporaries X0, X2, X3 and then the rows' reverse arrays are written (X2 also
  // holds the forward RNEA's forces, before A is formed); the Gauss-Seidel tape is dead after the reverse
  // Gauss-Seidel, when the reverse pass's per-link accumulators wr, sb, cb, tI are cleared
  L.J = take(rc * L.nvp);
  L.W = take(std::max(rc * L.nvp, 18 * nv));
  L.colS = L.W; L.colY = L.W + 6 * nv; L.colYv = L.W + 12 * nv;
  const int ntri = rc * (rc + 1) / 2;
  L.A = take(std::max({2 * ntri, 19 * rc, 18 * nl})); L.Ab = L.A + ntri;
  L.X0 = L.A; L.X2 = L.A + 6 * nl; L.X3 = L.A + 12 * nl;
  L.rxb = L.A; L.rdb = L.A + 3 * rc; L.rqb = L.A + 6 * rc; L.rwa = L.A + 7 * rc; L.rwb = L.A + 13 * rc;
  L.rbc = take(rc); L.rb = take(rc); L.rinvA = take(rc); L.rlam = take(rc); L.rybar = take(rc); L.rbbar = take(rc);
  L.rx = take(3 * rc); L.rcen = take(3 * rc); L.rd = take(3 * rc);
  L.hlo = take(std::max(2 * iters * L.rcp, 18 * nl)); L.hres = L.hlo + iters * L.rcp;
  L.wr = L.hlo; L.sb = L.hlo + 6 * nl; L.cb = L.hlo + 12 * nl; L.tI = L.hlo + 15 * nl;
  L.misc = take(8);
  L.n_real = (off + 1) & ~1;
  off = 0;
  L.rkind = take(rc); L.rlink = take(rc); L.rdof = take(rc); L.rnrm = take(rc); L.rmap = take(rc);
  L.rlinkb = take(rc); L.rslot = take(rc);
  L.hst = take(iters * L.rcp); L.flags = take(64);
  L.t_li = L.t_lev = L.t_links = L.t_child = L.t_col = L.t_dof = -1;
  if (stage_tables) {
    L.t_li = take(kLinkIntCols * nl); L.t_lev = take(nl + 1); L.t_links = take(nl); L.t_child = take(nl);
    L.t_col = take(nv); L.t_dof = take(nd);
  }
  L.n_int = off;
  return L;
}

}  // namespace ags
