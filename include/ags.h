/*
 * ags — batched articulated-body physics step for AMD MI355X (gfx950).
 *
 * C ABI of the hot path of the simulator described in "Isaac Gym: High Performance GPU-Based
 * Physics Simulation For Robot Learning" (arXiv 2108.10470): thousands of independent robot
 * environments, each a set of reduced-coordinate articulations (Section 3), advanced together on
 * one GPU with the physics state kept in flat device tensors (Section 2.3, Tables 1-2).
 *
 * Conventions
 *  - All tensors are float32, row-major, on the device, owned by the caller (e.g. PyTorch): the
 *    library reads and writes them in place ("zero-copy" tensor wrapping, Section 2.3.1).
 *  - Spatial quantities use z-up, ground plane z = 0, quaternions xyzw (actor root state columns
 *    0:3 position, 3:7 quaternion, 7:10 linear velocity, 10:13 angular velocity; Section 2.3.2).
 *    The position and linear velocity of a free root are those of its centre of mass: a free
 *    root link's frame must sit at its centre of mass (ags_model_create rejects it otherwise).
 *  - DOF units are radians (revolute) and metres (prismatic) (Section 2.3.2).
 *  - Environments are laid out env-major: env e's actors, DOFs and bodies are contiguous rows of
 *    the global tensors, in the order of its model's actors and their links.
 *  - Every call returns 0 on success or a negative AGS_E_* code; ags_last_error() returns a
 *    thread-local message for the last failure.  Calls that enqueue GPU work are asynchronous on
 *    the stream passed to them and never synchronise the host.
 *  - A sim is not thread-safe; different sims are independent.
 */
#ifndef AGS_H
#define AGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
enum {
  AGS_OK = 0,
  AGS_E_ARG = -1,      /* bad argument (null pointer, out-of-range index, unsupported size) */
  AGS_E_MODEL = -2,    /* inconsistent model description */
  AGS_E_HIP = -3,      /* HIP runtime error (message has the HIP error string) */
  AGS_E_NOMEM = -4,    /* device allocation failed */
  AGS_E_UNBOUND = -5   /* a tensor the call needs is not bound */
};
const char* ags_last_error(void);

/* ---------------------------------------------------------------- model description
 * An actor is an articulation: a tree of links with parent index < child index (Section 3;
 * "actor", "rigid bodies" and "DOF states", Section 2.2).  Joint types: the root link has a free
 * (floating-base) or fixed joint; every other link has a 1-DOF revolute or prismatic joint
 * (Section 2.2: fixed 0 DOF, revolute and prismatic 1 DOF; a spherical joint is expressed as a
 * chain of revolutes through massless links).  A rigid body is a one-link articulation. */
enum { AGS_JOINT_FREE = 0, AGS_JOINT_FIXED = 1, AGS_JOINT_REVOLUTE = 2, AGS_JOINT_PRISMATIC = 3 };
enum { AGS_SHAPE_SPHERE = 0, AGS_SHAPE_CAPSULE = 1, AGS_SHAPE_BOX = 2 };

typedef struct {
  int32_t parent;      /* actor-local parent link, -1 for the root */
  int32_t joint;       /* AGS_JOINT_* */
  float anchor[3];     /* joint origin in the parent link frame (link frames coincide with the parent's at q = 0) */
  float axis[3];       /* joint axis (normalised by the library) */
  float lower, upper;  /* DOF limits (+-INFINITY: none), enforced as unilateral constraint rows */
  float kp, kd;        /* PD drive stiffness and damping (Table 3 "drive stiffness/damping"), 0: no drive */
  float armature;      /* joint armature (Table 3) */
  float mass;          /* > 0: link mass (shapes then only give its distribution); 0: from shape densities */
} ags_link_desc;

typedef struct {
  int32_t link;        /* actor-local link */
  int32_t kind;        /* AGS_SHAPE_* */
  float p0[3];         /* sphere / box centre, or first capsule cap centre, in the link frame */
  float p1[3];         /* second capsule cap centre */
  float radius;        /* sphere / capsule radius */
  float half[3];       /* box half extents (box axes = link frame axes) */
  float density;       /* kg / m^3 */
} ags_shape_desc;

typedef struct {
  int32_t n_links, n_shapes;
  const ags_link_desc* links;
  const ags_shape_desc* shapes;
} ags_actor_desc;

/* Collision pair: shape a_shape of actor a_actor against the ground plane (b_actor = -1) or
 * against box b_shape of actor b_actor (a sphere or capsule vs a box of another actor).
 * Pairs never cross environments (Section 2.1: environments do not interact). */
typedef struct {
  int32_t a_actor, a_shape, b_actor, b_shape;
} ags_pair_desc;

typedef struct ags_model ags_model;

/* Compile one environment template (its actors and collision pairs).  Host-only; copies
 * everything it needs.  Limits: at most 64 links, 64 generalized velocities and 256 contact
 * slots per environment. */
int ags_model_create(const ags_actor_desc* actors, int32_t n_actors, const ags_pair_desc* pairs,
                     int32_t n_pairs, ags_model** out);
void ags_model_destroy(ags_model* model);

/* Fixed tendon (appendix on tendons: a mechanism coupling DOFs of one articulation).  A tree of n_joints
 * tendon joints, each following the incoming 1-DOF joint of link[j] (actor-local, not the root) with
 * coefficient coef[j]; parent[j] is its parent tendon joint (-1 for the root; parents listed first).  The
 * length at joint j is l_j = l_parent + coef[j] q_link[j].  At every tendon joint the force
 * f_j = stiffness (l_j - rest_length) + damping dl_j/dt, plus limit_stiffness (l_j - upper) above upper and
 * limit_stiffness (l_j - lower) below lower, acts on each DOF of the path from the tendon's root to j as
 * the generalized force -f_j coef.  Forces are explicit: evaluated at the state at the start of each
 * substep (stable while (stiffness + limit_stiffness) h^2 is small against the joints' effective
 * inertia).  The adjoint does not support models with tendons. */
typedef struct {
  int32_t actor, n_joints;
  const int32_t* link;
  const int32_t* parent;
  const float* coef;
  float stiffness, damping, rest_length, lower, upper, limit_stiffness;
} ags_tendon_desc;
/* Add fixed tendons to a model (before any sim is created from it).  Errors: AGS_E_ARG (bad pointers),
 * AGS_E_MODEL (actor, link or parent out of range, a root link, a parent listed after its child). */
int ags_model_add_tendons(ags_model* model, const ags_tendon_desc* tendons, int32_t n_tendons);

typedef struct {
  int32_t n_actors, n_links, n_dof, n_v, n_slots, max_rows;
} ags_model_info;
int ags_model_get_info(const ags_model* model, ags_model_info* out);

/* Per-link mass, COM (link frame) and inertia about the COM (link frame, 3x3 row-major), host
 * arrays of n_links, 3 n_links and 9 n_links floats. */
int ags_model_mass_props(const ags_model* model, float* mass, float* com, float* inertia);

/* ---------------------------------------------------------------- simulation
 * Parameters of Table 3 that the step uses.  One env-step advances dt with `substeps` substeps of
 * h = dt / substeps, the controls held over the step (Table 4: sim dt 1/120 s, control dt 1/60 s).
 * Contacts and limits are unilateral constraint rows solved by pgs_iters sweeps of projected
 * Gauss-Seidel ("position iterations"), with Coulomb friction mu (Table 3) and a Baumgarte
 * factor for penetration ("max bias coefficient"). */
typedef struct {
  float dt;
  int32_t substeps;
  float gravity[3];
  int32_t pgs_iters;
  float mu;
  float baumgarte;
  float contact_margin;     /* a contact row exists when phi + h min(0, v_n) < contact_margin */
  float limit_margin_rev;   /* same test for revolute limits (rad) */
  float limit_margin_pri;   /* and prismatic limits (m) */
  int32_t compute_fp64;     /* 0: compute in FP32; 1: compute in FP64 (tensors stay FP32) */
  int32_t lanes_per_env;    /* 0 or 64: one environment per 64-lane wavefront; 32: two environments per wavefront
                               (only for models with n_v <= 32) */
  int32_t persistent;       /* 1: one launch for all environment types (a grid sized to the device walks a work
                               list ordered by estimated cost, heaviest first); 0: one launch per type */
  int32_t adjoint_precision;  /* ags_sim_step_backward computes in: 0 the precision of compute_fp64, 32 FP32,
                                 64 FP64 */
  int32_t solver;           /* 0: projected Gauss-Seidel (AGS_SOLVER_PGS); 1: the temporal variant
                               (AGS_SOLVER_TGS, Section 3): the same rows and sweeps, but after every sweep
                               the velocity times h / pgs_iters is accumulated per row as J_r v, and each
                               contact-normal and limit row's bias is recomputed from its position error
                               plus that accumulated displacement.  The adjoint supports PGS only. */
  int32_t adjoint_max_rows; /* 0: 64; 1..64: constraint rows per substep the adjoint accepts (an environment
                               whose substep has more gets a zero adjoint and status 1); a smaller cap
                               shrinks the adjoint's LDS layout */
} ags_sim_params;

enum { AGS_SOLVER_PGS = 0, AGS_SOLVER_TGS = 1 };

typedef struct ags_sim ags_sim;

/* Create a batch of n_envs environments; env_model[e] (host array) indexes models[] and selects
 * the template of env e (heterogeneous batches allowed).  Allocates the device-side model tables
 * and scratch; tensors are bound separately. */
int ags_sim_create(const ags_model* const* models, int32_t n_models, const int32_t* env_model, int32_t n_envs,
                   const ags_sim_params* params, ags_sim** out);
void ags_sim_destroy(ags_sim* sim);

/* Tensor shapes (rows, cols) follow Tables 1-2:
 *   AGS_ROOT_STATE         (N_A, 13)  get/set  actor root states
 *   AGS_DOF_STATE          (N_D, 2)   get/set  DOF position, velocity
 *   AGS_DOF_ACTUATION      (N_D, 1)   control  DOF actuation forces (torques or forces)
 *   AGS_DOF_POS_TARGET     (N_D, 1)   control  PD position targets
 *   AGS_DOF_VEL_TARGET     (N_D, 1)   control  PD velocity targets
 *   AGS_NET_CONTACT_FORCE  (N_B, 3)   get      net contact force on each rigid body (world frame)
 *   AGS_DOF_FORCE          (N_D, 1)   get      force applied at each DOF (actuation + drive), step average
 *   AGS_RIGID_BODY_STATE   (N_B, 13)  get      rigid-body states after the step (Table 1): link-frame origin,
 *                          orientation quaternion xyzw, velocity of the origin, angular velocity (world)
 *   AGS_ENV_STATUS         (E, 1)  int32  get  per-env status of the last step: bit 0 the new state is not
 *                          finite, bit 1 a substep had more than 32 rows (or a Jacobian row too long for the
 *                          register form) and took one of the slower row paths (responses in chunks of 32
 *                          rows; with 64 lanes per env and up to 64 rows the Delassus columns are streamed
 *                          from scratch, otherwise rows and cross-lane sums); failures never fail the call
 *   AGS_DEBUG_QDD_FREE     (E, substeps * max n_v)       unconstrained joint accelerations per substep
 *   AGS_DEBUG_ROW_COUNT    (E, substeps)  int32          constraint rows per substep
 *   AGS_DEBUG_ROW_KEY      (E, substeps * max rows) int32  row keys (kind << 24 | a << 8 | b)
 *   AGS_DEBUG_ROW_LAMBDA   (E, substeps * max rows)      row impulses after the last sweep
 *   AGS_DEBUG_ADJ_CYCLES   (E, 11)  int64                shader-clock cycles per phase of ags_sim_step_backward
 *                          (recompute: other parts, Gauss-Seidel; reverse: Gauss-Seidel, dense products,
 *                          mass-matrix terms, RNEA, rows and wrenches, integration and solves; recompute:
 *                          composite inertias + dense M~ + its Cholesky factor, J rows + W = M~^-1 J^T,
 *                          Delassus A = J W^T on the matrix cores), for profiling
 *   AGS_DEBUG_PHASE_CYCLES (E, 10)  int64                shader-clock cycles per phase of the step (controls,
 *                          forward sweep, inward sweep, outward sweep, v* sweep, narrow phase, rows,
 *                          row responses, Gauss-Seidel, outputs), for profiling
 * Per-env physical properties (domain randomization, Section 2: copies of an environment may vary;
 * the paper's hand setup randomizes masses, friction, joint limits, drive gains and gravity).  When
 * bound they replace the model's or the parameters' value for each env; unbound, the model's apply.
 * Read by ags_sim_step and ags_sim_jacobian_mass (mass scale); ags_sim_step_backward refuses a sim with
 * any of them bound.
 *   AGS_BODY_MASS_SCALE    (N_B, 1)   factor on each link's mass and rotational inertia (COM unchanged)
 *   AGS_DOF_STIFFNESS      (N_D, 1)   drive kp of each DOF
 *   AGS_DOF_DAMPING        (N_D, 1)   drive kd of each DOF
 *   AGS_DOF_LIMITS         (N_D, 2)   lower, upper limit of each DOF (+-infinity: none)
 *   AGS_ENV_FRICTION       (E, 1)     friction coefficient mu of each env
 *   AGS_ENV_GRAVITY        (E, 3)     gravity vector of each env
 * Outputs and debug tensors are written only when bound.  N_A, N_D and N_B count actors, DOFs
 * and links of all environments. */
enum {
  AGS_ROOT_STATE = 0, AGS_DOF_STATE, AGS_DOF_ACTUATION, AGS_DOF_POS_TARGET, AGS_DOF_VEL_TARGET,
  AGS_NET_CONTACT_FORCE, AGS_DOF_FORCE, AGS_DEBUG_QDD_FREE, AGS_DEBUG_ROW_COUNT, AGS_DEBUG_ROW_KEY,
  AGS_DEBUG_ROW_LAMBDA, AGS_DEBUG_PHASE_CYCLES, AGS_DEBUG_ADJ_CYCLES, AGS_RIGID_BODY_STATE, AGS_ENV_STATUS,
  AGS_BODY_MASS_SCALE, AGS_DOF_STIFFNESS, AGS_DOF_DAMPING, AGS_DOF_LIMITS, AGS_ENV_FRICTION, AGS_ENV_GRAVITY,
  AGS_NUM_TENSORS
};
int ags_sim_tensor_shape(const ags_sim* sim, int32_t which, int64_t* rows, int64_t* cols);
/* Bind a device pointer (NULL unbinds).  The memory must hold rows x cols elements and stay valid
 * while steps that use it are in flight. */
int ags_sim_bind(ags_sim* sim, int32_t which, void* device_ptr);

/* One env-step of every environment, enqueued on hip_stream (a hipStream_t; NULL = default).
 * Reads and rewrites the bound root and DOF state tensors in place; needs ROOT_STATE, DOF_STATE
 * and DOF_ACTUATION bound (the PD target tensors are read only when bound; unbound targets are 0). */
int ags_sim_step(ags_sim* sim, void* hip_stream);

/* Reverse-mode derivative of one env-step (a hand-written adjoint; the paper's simulator is not
 * differentiable, this is the differentiation pattern of training systems built on such batched
 * steps).  Given the state at the START of a step (root_state (N_A,13), dof_state (N_D,2)), the
 * controls it used (actuation (N_D); the bound PD targets, if any, are read as in ags_sim_step) and
 * the adjoint of the state AFTER the step in root_adj / dof_adj (same shapes: dL/d of every state
 * entry), this call overwrites root_adj / dof_adj with the adjoint of the state before the step
 * and writes act_adj (N_D) = dL/d actuation of this step.  All pointers are device memory owned by
 * the caller; nothing is allocated.
 * The derivative is that of the smooth piece the state lies in: which rows exist, which bias
 * branch each row takes and which bound each Gauss-Seidel update clamps to are held at the values
 * the recomputed step takes (a mode switch is where the step is not differentiable).  Quaternion
 * adjoints are tangent to the unit sphere; the pose of a fixed root is a constant (its adjoint rows
 * come back zero); PD targets receive no adjoint.
 * Limits: at most 32 Gauss-Seidel sweeps, at most adjoint_max_rows (default 64) constraint rows per environment
 * and substep: an environment whose substep has more gets zero adjoints and status[env] = 1 (status: optional device int32 per
 * environment, 0 on success).  Computes in the precision chosen by adjoint_precision. */
int ags_sim_step_backward(ags_sim* sim, const float* root_state, const float* dof_state, const float* actuation,
                          float* root_adj, float* dof_adj, float* act_adj, int32_t* status, void* hip_stream);

/* Autotuner: picks the fastest mapping of environments onto wavefronts (lanes_per_env 64 or 32, the
 * latter only when every environment has at most 32 generalized velocities) and launch form
 * (persistent or per type) for this batch on the current device.  Each candidate sim is created,
 * stepped n_steps times twice (the first time warms up) from private device copies of root_state /
 * dof_state with the given actuation (device arrays shaped like the bound tensors), timed with HIP
 * events on hip_stream (the call synchronises that stream), and destroyed; the caller's arrays are
 * not modified.  On success params->lanes_per_env and params->persistent hold the winner and
 * *ms_out (optional) its milliseconds per env-step. */
int ags_autotune(const ags_model* const* models, int32_t n_models, const int32_t* env_model, int32_t n_envs,
                 ags_sim_params* params, const float* root_state, const float* dof_state, const float* actuation,
                 int32_t n_steps, float* ms_out, void* hip_stream);

/* Jacobian and generalized mass-matrix tensors (Section 2.3, Table 1: available for articulated actors,
 * per homogeneous group, for operational-space control and inverse kinematics) of the envs that use
 * models[model] (the index among the models the sim was created with), in increasing env id, at the
 * state in the bound root / DOF state tensors.  With nb = n_links and nv = n_v of that model
 * (ags_model_get_info) and n its env count:
 *   jac  (device, n x nb x 6 x nv, row-major): for every link (body) b of the env, rows 0-2 the world
 *        velocity of b's frame origin and rows 3-5 b's world angular velocity per unit rate of each
 *        generalized velocity column;
 *   mass (device, n x nv x nv): the joint-space inertia M(q) in the same columns (symmetric; armature
 *        not included), i.e. the kinetic energy is 1/2 qd^T M qd.
 * Columns: per actor in order, a free root's world COM velocity (3) and world angular velocity (3), then
 * the actor's joint rates; the columns of other actors of the env are zero for b.  Either output may be
 * NULL; the call only enqueues work on hip_stream.  Errors: AGS_E_ARG (no env uses the model, both outputs
 * NULL), AGS_E_UNBOUND (state tensors not bound). */
int ags_sim_jacobian_mass(ags_sim* sim, int32_t model, float* jac, float* mass, void* hip_stream);

/* Rollouts with checkpoints (the checkpoint-every-k recomputation pattern of differentiable
 * simulation).  A state is 13 N_A + 2 N_D floats: the root-state rows, then the DOF-state rows. */
int ags_rollout_state_size(const ags_sim* sim, int64_t* floats);
/* n_steps env-steps from the bound root/DOF state tensors (advanced in place to the final state) with
 * actions[t] = actions + t N_D (device, n_steps x N_D) as the control of step t: the actuation
 * (control = AGS_DOF_ACTUATION) or the PD position targets (control = AGS_DOF_POS_TARGET; the bound
 * actuation tensor then supplies the actuation of every step).  The state before every `every`-th step
 * (t = 0, every, 2 every, ...) is copied to ckpt (device, ceil(n_steps / every) states).  The bound
 * tensors are left as they were. */
int ags_rollout_forward(ags_sim* sim, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                        float* ckpt, void* hip_stream);
/* Reverse pass of a rollout made by ags_rollout_forward with the same n_steps, every, control, actions
 * and ckpt: root_adj / dof_adj hold dL/d(final state) on entry and dL/d(initial state) on return;
 * act_adj (device, n_steps x N_D) receives dL/d actions[t] (for PD targets, kp dL/d(joint force): the
 * target enters the step only through the drive force kp (q* - q - h qd)).  seg is caller-owned device
 * scratch of ags_rollout_seg_bytes(sim, every) bytes (two segment buffers): each segment is recomputed
 * from its checkpoint with ags_sim_step (output tensors untouched), keeping every step's substep states,
 * and its steps are reversed with ags_sim_step_backward, which then starts from those states instead of
 * recomputing them.  status (optional, device int32 per environment) is cleared by the call and set to 1
 * for every environment that exceeded the adjoint's row capacity at ANY step of the rollout (its zero
 * adjoint at that step also zeroes the gradients of all earlier steps).  The recomputation of the next
 * (earlier) segment runs on a second stream the sim owns, overlapping the current segment's adjoint;
 * events order the two buffers, and all work is joined into hip_stream before the call's last launch. */
int ags_rollout_seg_bytes(const ags_sim* sim, int32_t every, int64_t* bytes);
int ags_rollout_backward(ags_sim* sim, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                         const float* ckpt, void* seg, float* root_adj, float* dof_adj, float* act_adj,
                         int32_t* status, void* hip_stream);

/* ags_rollout_backward without the workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training or serving loops, harnesses that forbid allocation): the
 * two segment buffers live in a static device array of the library (64 MiB, one copy per GPU, held until
 * the process ends; its address on a device is taken when a sim is created there, as are the rollout's
 * streams, so this call creates, allocates and frees nothing).  Same arguments, results and status as
 * ags_rollout_backward, bit for bit.  Errors: AGS_E_ARG as there, and when 2 x one segment buffer (see
 * ags_rollout_seg_bytes) exceeds 64 MiB (4096 humanoid-like envs: checkpoint intervals up to 12; 4096
 * ant-like envs: up to 22).  Every call on one GPU uses the same array, which keeps the last call's
 * contents (each call writes every word before reading it, so nothing needs clearing): calls that overlap
 * on one GPU (two streams, two sims, two threads) race and must be serialised by the caller. */
int ags_rollout_backward_noalloc(ags_sim* sim, int32_t n_steps, int32_t every, int32_t control, const float* actions,
                                 const float* ckpt, float* root_adj, float* dof_adj, float* act_adj, int32_t* status,
                                 void* hip_stream);

/* Rollouts with a stored tape: the forward pass keeps everything the reverse pass needs, which then
 * recomputes nothing (the store-everything end of the checkpointing trade-off, for when memory allows:
 * about 660 B per humanoid env-step at two substeps).  The tape (device, caller-owned,
 * ags_rollout_tape_bytes(sim, n_steps) bytes, 256-byte aligned parts) holds the FP32 state before every
 * step, the FP64 state at the start of every non-first substep of every step, and a per-env flag of
 * steps with many constraint rows (which adjoint layout to use).  ags_rollout_forward_tape advances the
 * bound state tensors like ags_rollout_forward (same actions and control conventions, output tensors
 * written by every step); ags_rollout_backward_tape, with the same n_steps, control, actions and tape,
 * returns the same adjoints as ags_rollout_backward (root_adj / dof_adj in-out, act_adj, status as there), bit
 * for bit, since the stored states are the ones a recomputation would produce.  The tape is read only;
 * flagged envs' adjoints run on a stream the sim owns, joined into hip_stream after every step. */
int ags_rollout_tape_bytes(const ags_sim* sim, int32_t n_steps, int64_t* bytes);
int ags_rollout_forward_tape(ags_sim* sim, int32_t n_steps, int32_t control, const float* actions, void* tape,
                             void* hip_stream);
int ags_rollout_backward_tape(ags_sim* sim, int32_t n_steps, int32_t control, const float* actions,
                              const void* tape, float* root_adj, float* dof_adj, float* act_adj, int32_t* status,
                              void* hip_stream);

/* Copy rows of src (same shape as the bound tensor) into the bound root / DOF state tensor for the
 * actors listed in actor_idx (device int32 array of n global actor indices; NULL with n equal to the
 * total actor count = all actors; n = 0 sets nothing, whatever actor_idx is).
 * Setting a root teleports the actor without changing its DOF poses; setting DOFs leaves roots
 * unchanged (Section 2.3.2). */
int ags_sim_set_root_state_indexed(ags_sim* sim, const float* src, const int32_t* actor_idx, int32_t n,
                                   void* hip_stream);
int ags_sim_set_dof_state_indexed(ags_sim* sim, const float* src, const int32_t* actor_idx, int32_t n,
                                  void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
