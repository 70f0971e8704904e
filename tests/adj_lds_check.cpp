// Host-side replay of the adjoint kernel's LDS layout (built with -fsanitize=address,undefined by the test):
// for one model size and parameter set, every array of make_adj_layout is touched at every index the
// kernel's indexing can reach (the extent of each array as the kernel indexes it: per link, per column,
// per row up to the layout's row capacity, per Gauss-Seidel sweep up to the tape's sweeps), in heap buffers
// of exactly n_real reals and n_int ints, so any formula that runs past the layout fails under the
// sanitizer or the explicit checks.  Prints one JSON line (byte offsets of every array, the total LDS
// bytes in FP32 and FP64, and the arrays that start beyond 64 KiB) and exits nonzero on a violation.
//   adj_lds_check n_links n_v n_dof n_actors max_rows substeps iters row_cap stage_tables
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ags_adj_layout.h"

using namespace ags;

namespace {
int g_fail = 0;

struct Arr {
  const char* name;
  int off;   // element offset
  long use;  // elements the kernel indexes from off
  bool ints;
};

void touch(std::vector<double>& real, std::vector<int>& in, const Arr& a) {
  if (a.off < 0 || a.use < 0) {
    std::fprintf(stderr, "negative offset or extent: %s\n", a.name);
    g_fail = 1;
    return;
  }
  const long end = (long)a.off + a.use;
  const long cap = a.ints ? (long)in.size() : (long)real.size();
  if (end > cap) {
    std::fprintf(stderr, "%s: [%d, %ld) exceeds the %s region of %ld\n", a.name, a.off, end, a.ints ? "int" : "real", cap);
    g_fail = 1;
    return;
  }
  for (long k = a.off; k < end; ++k) {  // every index, through the buffer the sanitizer watches
    if (a.ints) in[k] += 1;
    else real[k] += 1.0;
  }
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 10) {
    std::fprintf(stderr, "usage: adj_lds_check n_links n_v n_dof n_actors max_rows substeps iters row_cap stage_tables\n");
    return 2;
  }
  ags_model_info info{};
  info.n_links = std::atoi(argv[1]);
  info.n_v = std::atoi(argv[2]);
  info.n_dof = std::atoi(argv[3]);
  info.n_actors = std::atoi(argv[4]);
  info.max_rows = std::atoi(argv[5]);
  const int substeps = std::atoi(argv[6]), iters = std::atoi(argv[7]), row_cap = std::atoi(argv[8]);
  const bool staged = std::atoi(argv[9]) != 0;
  const AdjLds L = make_adj_layout(info, substeps, iters, row_cap, staged);
  const int nl = info.n_links, nv = std::max(1, info.n_v), nd = std::max(1, info.n_dof), na = info.n_actors;
  const int rc = L.rows_cap, nvp = L.nvp, rcp = L.rcp;
  const long ntri = (long)rc * (rc + 1) / 2;
  if (rc < 1 || rc > row_cap || rc > kAdjRows || nvp < nv || rcp < rc || iters > kAdjIters) {
    std::fprintf(stderr, "bad layout parameters\n");
    return 1;
  }
  // extents as the kernel indexes them
  const std::vector<Arr> arrays = {
      // per link i < n_links: a fixed width each
      {"Rm", L.Rm, 9l * nl, false}, {"p", L.p, 3l * nl, false}, {"ax", L.ax, 3l * nl, false},
      {"c", L.c, 3l * nl, false}, {"Iw", L.Iw, 6l * nl, false}, {"Ic", L.Ic, 10l * nl, false},
      {"V", L.V, 6l * nl, false}, {"Vs", L.Vs, 6l * nl, false}, {"X1", L.X1, 6l * nl, false},
      // the RNEA's per-link temporaries, in A's words (A is dead while they live)
      {"X0", L.X0, 6l * nl, false}, {"X2", L.X2, 6l * nl, false}, {"X3", L.X3, 6l * nl, false},
      // the reverse pass's per-link accumulators, in the Gauss-Seidel tape's words (cleared after its last read)
      {"wr", L.wr, 6l * nl, false}, {"sb", L.sb, 6l * nl, false}, {"cb", L.cb, 3l * nl, false},
      {"tI", L.tI, 3l * nl, false},
      // per generalized velocity column
      {"nu", L.nu, nv, false}, {"qdd", L.qdd, nv, false}, {"vs", L.vs, nv, false}, {"nu1", L.nu1, nv, false},
      {"tau", L.tau, nv, false}, {"arm", L.arm, nv, false}, {"z", L.z, nv, false}, {"w", L.w, nv, false},
      {"nub", L.nub, nv, false}, {"vsb", L.vsb, nv, false}, {"nui", L.nui, nv, false}, {"tmp", L.tmp, nv, false},
      {"cs", L.cs, 6l * nv, false},
      // per DOF
      {"q", L.q, nd, false}, {"qb", L.qb, nd, false}, {"ab", L.ab, nd, false},
      // the start state of every substep and the end state (st + s * state_words, s <= substeps)
      {"st", L.st, (long)(substeps + 1) * L.state_words, false},
      {"rbar", L.rbar, 13l * na, false}, {"dbar", L.dbar, 2l * nd, false}, {"nrb", L.nrb, 13l * na, false},
      // packed lower triangle of the factor (then P): entry (i, j), j <= i < n_v, at i (i + 1) / 2 + j; the
      // reciprocal diagonal
      {"Lm", L.Lm, (long)nv * (nv + 1) / 2, false}, {"ldi", L.ldi, nv, false},
      // rows: J and W rows (row < rows_cap, column < n_v at stride nvp)
      {"J", L.J, (long)(rc - 1) * nvp + nv, false}, {"W", L.W, (long)(rc - 1) * nvp + nv, false},
      // mass-matrix column vectors, alive after W is dead, in W's words
      {"colS", L.colS, 6l * nv, false}, {"colY", L.colY, 6l * nv, false}, {"colYv", L.colYv, 6l * nv, false},
      // packed symmetric Delassus matrix and S = Abar + Abar^T (tri(s, r), s, r < rows_cap)
      {"A", L.A, ntri, false}, {"Ab", L.Ab, ntri, false},
      // per-row reverse arrays, alive after A and S are dead, in A's words
      {"rxb", L.rxb, 3l * rc, false}, {"rdb", L.rdb, 3l * rc, false}, {"rqb", L.rqb, rc, false},
      {"rwa", L.rwa, 6l * rc, false}, {"rwb", L.rwb, 6l * rc, false},
      {"rbc", L.rbc, rc, false}, {"rb", L.rb, rc, false}, {"rinvA", L.rinvA, rc, false}, {"rlam", L.rlam, rc, false},
      {"rybar", L.rybar, rc, false}, {"rbbar", L.rbbar, rc, false}, {"rx", L.rx, 3l * rc, false},
      {"rcen", L.rcen, 3l * rc, false}, {"rd", L.rd, 3l * rc, false},
      // Gauss-Seidel tape: hlo[it * rcp + r], it < iters, r < rows_cap
      {"hlo", L.hlo, (long)(iters - 1) * rcp + rc, false}, {"hres", L.hres, (long)(iters - 1) * rcp + rc, false},
      {"misc", L.misc, 8, false},
      // integer region
      {"rkind", L.rkind, rc, true}, {"rlink", L.rlink, rc, true}, {"rdof", L.rdof, rc, true},
      {"rnrm", L.rnrm, rc, true}, {"rmap", L.rmap, rc, true}, {"rlinkb", L.rlinkb, rc, true},
      {"rslot", L.rslot, rc, true}, {"hst", L.hst, (long)(iters - 1) * rcp + rc, true}, {"flags", L.flags, 64, true},
      // staged model tables: link table, level starts (a level has at least one link), links by level,
      // children (fewer than the links), link of each column and of each DOF
  };
  std::vector<Arr> all = arrays;
  if (staged)
    all.insert(all.end(), {{"t_li", L.t_li, (long)kLinkIntCols * nl, true}, {"t_lev", L.t_lev, nl + 1l, true},
                           {"t_links", L.t_links, nl, true}, {"t_child", L.t_child, nl, true},
                           {"t_col", L.t_col, nv, true}, {"t_dof", L.t_dof, nd, true}});
  std::vector<double> real((size_t)L.n_real, 0.0);
  std::vector<int> in((size_t)L.n_int, 0);
  for (const Arr& a : all) touch(real, in, a);
  // arrays that share words in time must stay inside their host array
  auto inside = [&](const char* what, long off, long use, long host, long host_words) {
    if (off < host || off + use > host + host_words) {
      std::fprintf(stderr, "%s leaves its host region\n", what);
      g_fail = 1;
    }
  };
  const long w_words = std::max((long)rc * nvp, 18l * nv), a_words = std::max({2 * ntri, 19l * rc, 18l * nl});
  const long t_words = std::max(2l * iters * rcp, 18l * nl);
  inside("colS", L.colS, 6l * nv, L.W, w_words);
  inside("colY", L.colY, 6l * nv, L.W, w_words);
  inside("colYv", L.colYv, 6l * nv, L.W, w_words);
  inside("Ab", L.Ab, ntri, L.A, a_words);
  inside("rxb..rwb", L.rxb, 19l * rc, L.A, a_words);
  inside("X0", L.X0, 6l * nl, L.A, a_words);
  inside("X2", L.X2, 6l * nl, L.A, a_words);
  inside("X3", L.X3, 6l * nl, L.A, a_words);
  inside("wr", L.wr, 6l * nl, L.hlo, t_words);
  inside("sb", L.sb, 6l * nl, L.hlo, t_words);
  inside("cb", L.cb, 3l * nl, L.hlo, t_words);
  inside("tI", L.tI, 3l * nl, L.hlo, t_words);
  inside("hres", L.hres, (long)(iters - 1) * rcp + rc, L.hlo, t_words);
  // arrays with their own words do not overlap: a word touched twice belongs to a shared region
  std::vector<int> owner((size_t)L.n_real, -1);
  for (size_t k = 0; k < arrays.size(); ++k) {
    const Arr& a = arrays[k];
    const std::string n = a.name;
    if (a.ints || n == "colS" || n == "colY" || n == "colYv" || n == "Ab" || n == "rxb" || n == "rdb" || n == "rqb" ||
        n == "rwa" || n == "rwb" || n == "X0" || n == "X2" || n == "X3" || n == "wr" || n == "sb" || n == "cb" ||
        n == "tI")
      continue;
    for (long i = a.off; i < a.off + a.use && i < L.n_real; ++i) {
      if (owner[i] >= 0) {
        std::fprintf(stderr, "%s overlaps %s at word %ld\n", a.name, arrays[owner[i]].name, i);
        g_fail = 1;
        break;
      }
      owner[i] = (int)k;
    }
  }
  std::vector<int> iowner((size_t)L.n_int, -1);
  for (size_t k = 0; k < all.size(); ++k) {
    const Arr& a = all[k];
    if (!a.ints) continue;
    for (long i = a.off; i < a.off + a.use && i < L.n_int; ++i) {
      if (iowner[i] >= 0) {
        std::fprintf(stderr, "%s overlaps %s at int %ld\n", a.name, all[iowner[i]].name, i);
        g_fail = 1;
        break;
      }
      iowner[i] = (int)k;
    }
  }
  const long bytes32 = 4l * L.n_real + 4l * L.n_int, bytes64 = 8l * L.n_real + 4l * L.n_int;
  std::printf("{\"rows_cap\": %d, \"n_real\": %d, \"n_int\": %d, \"bytes_f32\": %ld, \"bytes_f64\": %ld, \"above_64KiB_f64\": [",
              rc, L.n_real, L.n_int, bytes32, bytes64);
  bool first = true;
  for (const Arr& a : all) {
    const long b = a.ints ? 8l * L.n_real + 4l * a.off : 8l * a.off;
    if (b + (a.ints ? 4 : 8) * (a.use > 0 ? a.use : 1) > 65536) {
      std::printf("%s\"%s\"", first ? "" : ", ", a.name);
      first = false;
    }
  }
  std::printf("], \"ok\": %s}\n", g_fail ? "false" : "true");
  return g_fail;
}
