// Internal layout shared by the host side and the HIP kernels of libags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ags_adj_layout.h"

namespace ags {

constexpr int kTeam = 64;       // lanes per environment: one wavefront
constexpr int kMaxLinks = 64;
constexpr int kMaxV = 64;       // generalized velocities per environment (one lane each in the solver)
constexpr int kMaxSlots = 256;
constexpr float kMinRowMass = 1e-6f;  // rows with J M~^-1 J^T below this are dropped (immovable)
constexpr int kPhases = 10;           // controls, forward, inward, outward, v*, narrow, rows, responses, PGS, outputs
constexpr int kJointEntries = 10;     // joint (non-root) entries of a compact Jacobian row
constexpr int kFastRows = 32;         // rows solved in registers (one per lane); also the row-response chunk

// per-link integer table
enum { LI_PARENT = 0, LI_JTYPE, LI_COL, LI_DOF, LI_ROOT, LI_CHILD_BEGIN, LI_CHILD_END, LI_ANC_BEGIN, LI_ANC_END,
       LI_ROOTCOL, LI_COLS };
// per-link float table (link frame quantities)
enum { LF_ANCHOR = 0, LF_AXIS = 3, LF_MASS = 6, LF_COM = 7, LF_IC = 10 /* xx yy zz xy xz yz */,
       LF_LO = 16, LF_HI, LF_KP, LF_KD, LF_ARM, LF_ML, LF_COLS };
// per-slot tables
enum { SLOT_SPHERE_PLANE = 0, SLOT_CORNER_PLANE = 1, SLOT_SPHERE_BOX = 2 };
enum { SI_TYPE = 0, SI_LINK_A, SI_LINK_B, SI_KEY, SI_COLS };
enum { SF_P = 0, SF_R = 3, SF_BOXC = 4, SF_HALF = 7, SF_COLS = 10 };
// per-actor table
enum { AI_ROOT = 0, AI_FIXED, AI_COL, AI_COLS };
// joint types (same numbering as the public header)
enum { J_FREE = 0, J_FIXED = 1, J_REV = 2, J_PRI = 3 };

// LDS layout of one environment's workgroup, offsets in 4-byte words
struct Lds {
  // integer model tables staged once per workgroup (the float tables stay in global memory)
  int t_li, t_lev, t_links, t_child, t_anc, t_dof, t_ai;
  // per environment, compute-type word offsets relative to its region; int arrays are packed
  int qj, qd, root, F;                 // state carried across substeps, summed contact forces
  int L0, vs;                          // per actor: root Cholesky factor (21) + 1/diag (6); per column: qdd, then v*
  int o, ax, U, Dinv, Ubar, G;         // per link (Ubar: angular half of U moved to the root), per ancestor pair
  int phi, n, x, sact;                 // per slot (sact: activity, then first row of the slot or -1)
  int rkr, rbias, rinvA, rlam;         // per row (rkr: kind << 16 | DOF or slot)
  int misc;                            // a few ints
  int q, v, IA, pA, u, tau, arm;       // dynamics region, dead after the narrow phase (pA then holds accelerations) ...
  int W, wstride;                      // ... shared with TEAM-row chunks of W
  int team_base, team_stride;          // per-environment region: base + team * stride
  int total;                           // words for all teams of a workgroup
};

struct DevModel {
  int n_links, n_actors, n_dof, n_v, n_slots, n_levels, n_anc, r_cap, n_body_slot;
  int jfast;  // every contact row's Jacobian fits the compact register form (kJointEntries joint entries)
  const int* li;
  const double* lf;
  const int* level_begin;
  const int* level_links;
  const int* children;
  const int* anc_link;
  const int* dof_link;   // link of each env DOF
  const int* si;
  const double* sf;
  const int* body_slot_begin;  // CSR per link: entries 2*slot + (1 if the link is side b)
  const int* body_slot;
  const int* ai;
  const unsigned long long* link_anc;  // per link: bit j set iff link j is an ancestor of it or itself
  const unsigned long long* col_anc;   // per column: bit j set iff column j precedes it on its path to the root
  const int* col_link;                 // per column: the link that owns it
  // fixed tendons: n_tj tendon joints (4 ints each: tendon, DOF, column, parent joint or -1; coefficient),
  // 6 doubles per tendon (stiffness, damping, rest length, lower, upper, limit stiffness)
  int n_tj;
  const int* tj_i;
  const double* tj_f;
  const double* tp;
};

// one environment type of a step launch: its model tables, LDS layout, environments and scratch
struct TypeArgs {
  DevModel m;
  Lds lds;
  const int* env_list;
  int n_envs;
  void* scratch;           // per env: J rows then W rows, r_cap x n_v each, in the compute type
  long long scratch_stride;
};

struct StepArgs {
  TypeArgs ty;  // the type of a per-type launch (unused by the fused launch)
  const int* env_actor_base;
  const int* env_dof_base;
  const int* env_body_base;
  float* root_state;
  float* dof_state;
  const float* act;
  const float* pos_tgt;
  const float* vel_tgt;
  float* contact_force;
  float* rb_state;  // optional (N_B, 13): link origin, quaternion, origin velocity, angular velocity
  int* env_status;  // optional (E): bit 0 non-finite new state, bit 1 row-response slow path taken
  int* big_rows;    // optional (E): 1 where a substep had more than kAdjBigRowsAt rows (adjoint layout hint)
  int* env_rows;    // optional (E): the most rows of a substep of the step (dispatch order of the next step)
  // optional per-env properties replacing the model's: link mass / inertia factor (N_B), drive kp, kd (N_D),
  // limits (N_D x 2), friction (E), gravity (E x 3)
  const float* mass_scale;
  const float* dof_kp;
  const float* dof_kd;
  const float* dof_limits;
  const float* env_mu;
  const float* env_gravity;
  float* dof_force;
  float* dbg_qdd;
  int dbg_qdd_stride, dbg_qdd_sub;  // per env, per substep (sim-wide maximum n_v)
  int* dbg_rc;
  int* dbg_key;
  float* dbg_lam;
  int dbg_row_stride, dbg_row_sub;  // per env, per substep (sim-wide maximum rows)
  long long* dbg_cycles;            // per env: shader-clock cycles spent in each phase (kPhases)
  // optional: the state after every substep but the last (FP64, the layout of a state: root rows then
  // DOF rows; block s of mid_block doubles holds substep s)
  double* mid_root;
  double* mid_dof;
  long long mid_block;
  double dt, h, gx, gy, gz, mu, beta, mc;
  int substeps, iters;
  int solver;  // 0 projected Gauss-Seidel, 1 temporal variant
};

// One launch over every environment type: a grid sized to the device walks a work list of
// (type, environment group) units ordered by estimated cost, heaviest first.
constexpr int kMaxFusedTypes = 4;
struct FusedArgs {
  StepArgs base;
  TypeArgs types[kMaxFusedTypes];
  const int* units;  // 2 ints per unit: type, group
  int n_units;
};
hipError_t launch_step_fused(const FusedArgs& a, int grid, size_t lds_bytes, int fp64, int team, hipStream_t stream);
hipError_t set_fused_lds_limit(int fp64, int team, size_t bytes);
hipError_t fused_blocks_per_cu(int fp64, int team, size_t lds_bytes, int* blocks);

// ---------------------------------------------------------------- Jacobian and mass-matrix tensors
struct JacMassArgs {
  DevModel m;
  const int* env_list;  // the envs of one model type (output entry i is env_list[i])
  int n_envs;
  const int* env_actor_base;
  const int* env_dof_base;
  const float* root_state;
  const float* dof_state;
  float* jac;   // optional: n_envs x n_links x 6 x n_v
  float* mass;  // optional: n_envs x n_v x n_v
  const int* env_body_base;
  const float* mass_scale;  // optional (N_B): per-link factor on mass and inertia
};
size_t jacmass_lds_bytes(int n_links, int n_v);
hipError_t launch_jacmass(const JacMassArgs& a, hipStream_t stream);

// ---------------------------------------------------------------- adjoint of one env-step
struct AdjArgs {
  DevModel m;
  AdjLds L;
  const int* env_list;
  const int* env_actor_base;
  const int* env_dof_base;
  const float* root_state;
  const float* dof_state;
  const float* act;
  const float* pos_tgt;
  const float* vel_tgt;
  float* root_adj;
  float* dof_adj;
  float* act_adj;
  int* status;
  int status_sticky;  // 0: status[env] = 0 or 1; 1: only failures are written (status kept across a rollout's steps)
  long long* cycles;  // optional, per env: kAdjPhases shader-clock counters
  const double* mid_root;  // optional: substep start states from the forward step (see StepArgs)
  const double* mid_dof;
  long long mid_block;
  int* retry;              // optional: environments whose rows exceed this layout's capacity are appended here
  int* retry_count;        //   (count at *retry_count) instead of being written with a zero adjoint
  const int* list_count;   // optional: number of valid entries of env_list (device), for a launch over a retry list
  const int* skip_flags;   // optional (indexed by env): envs whose flag is set are left to another launch
  double h, gx, gy, gz, mu, beta, mc;
  int substeps, iters;
};

// grid in (0, n_envs): that many workgroups stride over a device list (a.list_count required);
// default: one workgroup per entry
hipError_t launch_adjoint(const AdjArgs& a, int n_envs, int fp64, hipStream_t stream, int grid = 0);
// list[0] (zeroed beforehand) = count, list[1 ...] = the envs of env_list[0, n) with flags[env] != 0
hipError_t launch_compact_flags(const int* env_list, int n, const int* flags, int* list, hipStream_t stream);
hipError_t set_adjoint_lds_limit(int fp64, size_t bytes);
hipError_t launch_zero_count(int* c, hipStream_t stream);
hipError_t launch_fill_int(int* p, int n, int value, hipStream_t stream);

hipError_t launch_scale_by_kp(float* x, const float* kp, int n, hipStream_t stream);

hipError_t launch_step(const StepArgs& a, int n_envs, int fp64, int team, hipStream_t stream);
// reorders the env ids order[0, n) by rows[env], most first (tmp: n ints)
hipError_t launch_order_by_rows(int* order, int* tmp, const int* rows, int n, hipStream_t stream);
hipError_t set_lds_limit(int fp64, int team, size_t bytes);
hipError_t launch_set_rows(float* dst, const float* src, const int* idx, int n, int n_actors, const int* table,
                           int field, int width, hipStream_t stream);

}  // namespace ags
