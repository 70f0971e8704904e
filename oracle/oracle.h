/*
 * FP64 CPU oracle for the batched articulated-physics step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of
 * bench.py may load this library.  It shares no code with the HIP library.
 *
 * Rigid-body dynamics follow the textbook definitions (Featherstone, "Rigid Body Dynamics
 * Algorithms", 2008): RNEA for the bias forces C(q, qd) (ch. 5), CRBA for the joint-space
 * inertia M(q) (ch. 6), dense Cholesky for M~ qdd = tau - C, and an ABA (ch. 7) kept only as a
 * self-check.  The paper (Section 3) names reduced-coordinate articulations, the sim
 * parameters of Table 3 and a Gauss-Seidel-family solver; the solver here is the
 * fixed-iteration projected Gauss-Seidel the hot path uses, reproduced step by step.
 *
 * Tables are row-major float64 arrays with the column layouts below.
 */
#ifndef AGS_ORACLE_H
#define AGS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* link table columns (one row per link, actors' links contiguous, actor-local parent index) */
enum {
  ORC_L_ACTOR = 0, ORC_L_PARENT, ORC_L_JOINT, /* joint: 0 free root, 1 fixed root, 2 revolute, 3 prismatic */
  ORC_L_ANCHOR, ORC_L_AXIS = ORC_L_ANCHOR + 3, ORC_L_LOWER = ORC_L_AXIS + 3, ORC_L_UPPER,
  ORC_L_KP, ORC_L_KD, ORC_L_ARMATURE, ORC_L_MASS, ORC_L_COLS
};
/* shape table columns */
enum {
  ORC_S_ACTOR = 0, ORC_S_LINK, ORC_S_KIND, /* kind: 0 sphere, 1 capsule, 2 box */
  ORC_S_P0, ORC_S_P1 = ORC_S_P0 + 3, ORC_S_RADIUS = ORC_S_P1 + 3, ORC_S_HALF, ORC_S_DENSITY = ORC_S_HALF + 3,
  ORC_S_COLS
};
/* pair table: 6 ints per pair: a_actor, a_link, a_shape(global row), b_actor (-1 plane), b_link, b_shape */
/* params vector */
enum {
  ORC_P_DT = 0, ORC_P_SUBSTEPS, ORC_P_GX, ORC_P_GY, ORC_P_GZ, ORC_P_ITERS, ORC_P_MU, ORC_P_BETA,
  ORC_P_MC, ORC_P_ML_REV, ORC_P_ML_PRI, ORC_P_GUARD_C, ORC_P_GUARD_L,
  ORC_P_SOLVER, /* 0 projected Gauss-Seidel, 1 its temporal variant (TGS) */
  ORC_P_COLS
};
/* row key: kind * 2^24 + a * 2^8 + b; kind 1 lower limit / 2 upper limit (a = env DOF index),
 * 3 contact normal / 4 tangent 1 / 5 tangent 2 (a = pair index, b = slot index) */

/* near-switch flag bits (per env, per substep).  ORC_NEAR_CLAMP: some Gauss-Seidel update's unclamped
 * impulse lies within 1e-6 (1 + |bound|) of a bound it is projected onto; the projection is continuous, so
 * this flag marks a switch of the step's derivative, not a jump of its value */
enum {
  ORC_NEAR_CONTACT = 1, ORC_NEAR_LIMIT = 2, ORC_NEAR_GEOM = 4, ORC_NEAR_SKIP = 8, ORC_NEAR_TANGENT = 16,
  ORC_NEAR_CLAMP = 32
};

void* orc_env_create(int n_actors, int n_links, const double* links, int n_shapes, const double* shapes,
                     int n_pairs, const int* pairs, char* err, int errlen);
void orc_env_destroy(void* env);
/* fixed tendons (appendix on tendons): params n_tendons x 6 (stiffness, damping, rest length, lower, upper,
 * limit stiffness); joints n_joints x 4 (tendon, env DOF index, parent tendon joint within the tendon or -1,
 * coefficient), each tendon's joints in tree order (a parent before its children) */
void orc_env_set_tendons(void* env, int n_tendons, const double* params, int n_joints, const double* joints);
/* sizes: out[0]=n_dof, [1]=n_v, [2]=n_bodies, [3]=n_actors, [4]=max rows per substep, [5]=n_slots */
void orc_env_sizes(const void* env, int* out);

/* per-body mass, COM (link frame) and rotational inertia about the COM (link frame, 3x3) */
void orc_mass_props(const void* env, double* mass, double* com, double* inertia);

/* world pose of every link: rotation (3x3 row-major, link->world) and origin */
void orc_fk(const void* env, const double* root_state, const double* dof_state, double* R, double* p);
/* Rigid-body states of one env (Table 1 "rigid body states"): per body (link), 18 values: origin of the
 * link frame (3), its rotation to world (9, row-major), the world velocity of the link origin (3) and the
 * world angular velocity (3), from the spatial velocities v_i = X_i v_parent + S_i qd_i. */
void orc_body_states(const void* env, const double* root_state, const double* dof_state, double* out);

/* joint-space quantities of one env: M (n_v x n_v, without armature), C (RNEA with qdd = 0, gravity
 * from params), qdd from CRBA+Cholesky and from ABA for generalized force tau (n_v), model armature only */
int orc_dynamics(const void* env, const double* params, const double* root_state, const double* dof_state,
                 const double* tau, double* M, double* C, double* qdd_crba, double* qdd_aba);

/* contact slots of one env state: per slot phi, normal, point, body a, body b (env body index, -1 plane) */
int orc_slots(const void* env, const double* root_state, const double* dof_state, double* phi, double* normal,
              double* point, int* body_a, int* body_b);

/* one env-step (params substeps) for n_envs envs; arrays are per-env contiguous.
 * root_in/out (n_envs, n_actors, 13); dof_in/out (n_envs, n_dof, 2); act/pos_tgt/vel_tgt (n_envs, n_dof);
 * qdd_free (n_envs, substeps, n_v); row_count (n_envs, substeps); row_key/row_lambda
 * (n_envs, substeps, r_cap); contact_force (n_envs, n_bodies, 3); dof_force (n_envs, n_dof);
 * contact_scale (n_envs, n_bodies, 2): per body, over the step's substeps, the number of contact rows
 * acting on it (either side) and the sum of their |impulse| / dt (the scale of its net contact force);
 * near (n_envs, substeps); mode (n_envs): a hash of every discrete decision of the step (row keys, the
 * bias branch of each row, the clamp taken by each Gauss-Seidel update), equal for two inputs exactly when
 * they lie in the same smooth piece of the step (up to hash collisions).  Output pointers may be NULL.
 * Returns 0 or -1 on a bad argument. */
int orc_step(const void* env, const double* params, int n_envs, const double* root_in, const double* dof_in,
             const double* act, const double* pos_tgt, const double* vel_tgt, double* root_out, double* dof_out,
             double* qdd_free, int r_cap, int* row_count, int* row_key, double* row_lambda,
             double* contact_force, double* contact_scale, double* dof_force, int* near, unsigned long long* mode,
             int n_threads);

#ifdef __cplusplus
}
#endif
#endif
