/*
 * mfm.h -- C ABI of the MI355X (gfx950) meshless finite-mass hydro pass.
 *
 * The method is the Lagrangian mesh-free finite-volume Godunov scheme that
 * Hopkins (2017), "A New Public Release of the GIZMO Code", names in its
 * abstract and in its "Arbitrary (Moving) Meshes" section: a gas sampled by
 * particles whose kernel-defined volumes are the cells of a mesh that moves
 * with the fluid, so mass is carried exactly and only momentum and energy
 * cross the faces between neighbours.  The paper gives no formulas; the pass
 * implements the standard finite-mass discretisation it refers to, in the
 * readings listed with each call below.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All particle arrays are DEVICE memory owned by the caller (allocated,
 *    e.g., through PyTorch).  The library never frees or reallocates them.
 *  - Arrays are structure-of-arrays FP64.  Multi-component arrays are
 *    component-major: component c of particle i sits at [c * n + i].
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL means the null stream).  Device-side conditions (no
 *    convergence, ill-conditioned E, neighbour-list overflow, non-finite
 *    results) are recorded in device counters and surface through
 *    mfm_check() / mfm_get_counters(), which synchronise the stream.
 *  - A call returns MFM_OK once its kernels are queued, or an error status
 *    after validating its arguments on the host, in which case nothing was
 *    launched.  mfm_last_error() gives a message.
 *  - The context owns only scratch memory sized at creation for `capacity`
 *    particles.  A call with n > capacity fails with MFM_E_CAPACITY.
 *  - Contexts are not thread-safe; calls that overlap on one context race.
 */
#ifndef MFM_H
#define MFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfm_ctx mfm_ctx;

typedef enum {
    MFM_OK = 0,
    MFM_E_INVALID = -1,    /* bad argument or parameter                         */
    MFM_E_HIP = -2,        /* a HIP runtime call failed                         */
    MFM_E_NOCONV = -3,     /* kernel-length iteration did not converge          */
    MFM_E_ILLCOND = -4,    /* gradient matrix singular or cond > cond_max       */
    MFM_E_MINIMAGE = -5,   /* a kernel length reached half a periodic box side  */
    MFM_E_CAPACITY = -6,   /* n > capacity, or a neighbour list overflowed      */
    MFM_E_NONFINITE = -7,  /* a NaN/Inf appeared in an output                   */
    MFM_E_STATE = -8       /* call order violated (e.g. pass before neighbours) */
} mfm_status;

typedef enum { MFM_FP64 = 0, MFM_MIXED = 1 } mfm_precision;

/* MFM: faces carry no mass (the Lagrangian form the rest of this header
 * describes).  MFV (the other mesh-free Godunov form that section 2 lists;
 * section 4 on meshes that move): the same pass, but the full HLLC flux of
 * mass, momentum and energy crosses each face, which moves with the mean
 * particle velocity, so masses change at the rate dm.  MFV runs in both
 * precisions; mfm_step integrates both forms and the adjoints accept only MFM. */
typedef enum { MFM_SCHEME_MFM = 0, MFM_SCHEME_MFV = 1 } mfm_scheme;

typedef struct {
    double gamma;          /* adiabatic index, > 1                                     */
    double n_ngb;          /* effective neighbour number, > 32/3                       */
    double cfl;            /* Courant factor of mfm_step when dt <= 0                  */
    double box[3];         /* box sides; positions must lie in [0, box)               */
    int32_t periodic[3];   /* 1: periodic (minimum image), 0: open                     */
    int32_t precision;     /* mfm_precision                                            */
    double beta;           /* slope-limiter constant (1 = Barth-Jespersen)             */
    double cond_max;       /* flag E when ||E||_F ||E^-1||_F exceeds this              */
    double u_floor;        /* floor on specific internal energy in mfm_step            */
    int32_t h_maxit;       /* cap on kernel-length iterations (<= 0: 64)               */
    int32_t max_ngb;       /* flux-list slots per particle (<= 0: 256)                 */
    int32_t tree_levels;   /* cell-table depth (<= 0: from n)                          */
    int32_t scheme;        /* mfm_scheme                                               */
    int32_t limiter;       /* 0: per-particle limiter only (R10, first order on a
                              non-positive face state, R12); 1: also the pairwise
                              face limiter (R23) and a condition-adaptive beta (R24) */
    double beta_min;       /* R24: limiter constant at cond(E) >= cond_hi               */
    double cond_lo;        /* R24: beta applies at cond(E) <= cond_lo                   */
    double cond_hi;        /* R24: between the two, beta moves linearly in log10(cond)  */
} mfm_params;

/*
 * One particle set, all device pointers, length n.  Inputs of the pass are
 * x, y, z, m, vx, vy, vz, u (and H as a guess).  Outputs are written by the
 * call named in brackets.  Pointers marked "nullable" may be NULL.
 */
typedef struct {
    int64_t n;
    double *x, *y, *z;       /* positions in [0, box)                               */
    double *m;               /* masses (constant under MFM; MFV steps update them)  */
    double *vx, *vy, *vz;    /* velocities                                          */
    double *u;               /* specific internal energy                            */
    double *H;               /* kernel support radius: in guess (<=0: cold), out root [solve_h] */
    double *nk;              /* kernel number density n_i           [solve_h]       */
    double *V;               /* volume 1/n_i                        [solve_h]       */
    double *B;               /* 6 x n: E^-1 as xx, xy, xz, yy, yz, zz  [gradients]  */
    double *rho, *P;         /* density m n, pressure (gamma-1) rho u  [gradients]  */
    double *grad;            /* 15 x n: limited gradients of rho, vx, vy, vz, P,
                                component-major (row 3 f + c)     [gradients]      */
    double *alpha;           /* nullable, 5 x n: limiter factors    [gradients]      */
    double *dp;              /* 3 x n: momentum rate dp/dt          [hydro_fluxes]   */
    double *dE;              /* total-energy rate dE/dt             [hydro_fluxes]   */
    double *vsig;            /* signal speed                        [hydro_fluxes]   */
    int64_t *id;             /* nullable: carried along every reordering            */
    double *dm;              /* mass rate dm/dt, MFV only (nullable, not written, under MFM) [hydro_fluxes] */
} mfm_particles;

typedef struct {
    int64_t pairs;           /* unordered flux pairs of the last hydro_fluxes       */
    int64_t list_entries;    /* directed flux-list entries (= 2 pairs)              */
    int64_t list_max;        /* longest flux list                                   */
    int64_t h_iters;         /* kernel-length iterations, summed                    */
    int64_t h_iters_max;     /* longest kernel-length iteration                     */
    int64_t noconv;          /* particles without a converged kernel length         */
    int64_t minimage;        /* particles whose radius reached half a periodic side */
    int64_t overflow;        /* particles whose flux list exceeded max_ngb          */
    int64_t illcond;         /* particles with det E <= 0 or cond > cond_max        */
    int64_t fallbacks;       /* directed pair evaluations that fell to first order  */
    int64_t clamps;          /* directed pair evaluations with P* clamped to 0      */
    int64_t nonfinite;       /* non-finite outputs                                  */
    int64_t floors;          /* u floors applied by mfm_step                        */
    int64_t first_bad;       /* lowest particle index flagged by any of the above   */
    double cond_max_seen;    /* largest ||E||_F ||B||_F                             */
    int64_t h_rounds_max;    /* most neighbour scans one kernel-length solve needed */
    int64_t h_fallback;      /* particles solved one wave each after the group scan */
    int64_t h_rounds3;       /* particles whose solve needed three or more scans    */
    int64_t gather_entries;  /* gather-set entries of the last solve_h, self excluded */
    int64_t h_rescan;        /* particles the rescanning kernel-length solver took   */
} mfm_counters;

/* Create a context for up to `capacity` particles.  Validates params:
 * gamma > 1, n_ngb > 32/3, box > 0, beta > 0, scheme MFM or MFV, limiter 0 or
 * 1 (with limiter 1: beta_min > 0 and 0 < cond_lo < cond_hi).  Allocates
 * scratch on the current HIP device.  *out is NULL on failure. */
mfm_status mfm_create(const mfm_params *params, int64_t capacity, mfm_ctx **out);

/* Free the context's scratch (synchronises its device).  NULL is a no-op. */
void mfm_destroy(mfm_ctx *ctx);

/* Neighbour structure (reading R2: gather set r < H_i, flux set
 * r < max(H_i, H_j); the search is the library's own choice).
 * Quantises positions to a per-axis Morton key, sorts particles by key
 * (stable LSD radix sort), REORDERS IN PLACE every non-NULL array among
 * x, y, z, m, vx, vy, vz, u, H, dp, dE, vsig, dm, id into that order, and
 * builds the per-level cell tables of the implicit octree.  Other output
 * arrays are left stale and are rewritten by the next pass. */
mfm_status mfm_build_neighbours(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* Undo the library's reorderings: puts the particles back in the order the
 * caller gave them in, for callers that want their results in that order.
 * Particle k moves to position id[k] in every non-NULL array of p (all rows
 * of B, grad, alpha and dp), so that afterwards id[i] = i.  id is required
 * (MFM_E_INVALID if NULL) and must hold every value 0 .. n-1 exactly once,
 * as it does if the caller set id[i] = i before the first reordering call;
 * the call checks this on the device and synchronises the stream once, and
 * returns MFM_E_INVALID with nothing moved if it does not.
 * The values are moved bit for bit.  Arrays outside p, such as the bins of
 * mfm_step_hier, are the caller's to move alike (new[id[k]] = old[k], with
 * id as it stood before the call).  The context's cell tables, lists and
 * per-level rates belong to the old order afterwards: the passes then
 * return MFM_E_STATE until mfm_build_neighbours runs, and the next
 * mfm_step_hier starts with a full pass. */
mfm_status mfm_unpermute(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* Kernel length (readings R1, R3-R5): H_i is the unique root of
 * (4 pi/3) H^3 n_i(H) = n_ngb, n_i(H) = sum_{r_ij < H} W(r_ij, H) with the
 * cubic spline of support H; nk = n_i(H_i), V = 1/nk.  FP64 in both
 * precisions.  H in: a guess (<= 0: from the local cell density).
 * Requires mfm_build_neighbours on the current positions.  Also builds each
 * particle's gather list (r < H_i, self excluded), which mfm_gradients
 * completes into the flux list (r < max(H_i, H_j)) used by mfm_hydro_fluxes. */
mfm_status mfm_solve_h(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* Gradients (readings R5-R8, R10): rho = m nk, P = (gamma-1) rho u;
 * E_i = sum_j d_ij d_ij^T W(r_ij, H_i) V_i over the gather set;
 * B = E^-1 (FP64 adjugate); least-squares gradients of rho, v, P limited per
 * particle by alpha = min(1, beta min((max-phi)/(|g| d), (phi-min)/(|g| d))),
 * d = half the largest gather distance.  Requires mfm_solve_h.
 * MFM_MIXED: the pairwise kernel weights W are FP32; the moments E, the
 * gradient sums and the inverse stay FP64; the per-particle record that the
 * flux kernel reads (state, B, limited gradients) is stored in FP32.
 * limiter = 1 (reading R24): beta is replaced per particle by
 * beta + (beta_min - beta) t, t = 0 at cond(E) <= cond_lo, 1 at >= cond_hi
 * (and for a singular E), linear in log10(cond) between. */
mfm_status mfm_gradients(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* Fluxes (readings R9, R11-R16, R18): per unordered pair in canonical order
 * (lower index is the left state): face A_ij = (V_i^2 W_i B_i + V_j^2 W_j B_j) d_ij,
 * midpoint linear reconstruction (first order if not positive), face frame
 * moving with the mean particle velocity, HLLC star state with Davis speeds,
 * zero mass flux, momentum P* A, energy P* (S* + w.n)|A|, applied with
 * opposite signs to both particles.  vsig_i = max_j [c_i + c_j
 * - min(0, (v_i - v_j).(x_i - x_j)/r)].  Requires mfm_gradients.
 * MFM_MIXED: displacements from FP64 positions, then kernel weights, faces,
 * reconstruction and HLLC in FP32; the per-particle sums of dp and dE in FP64.
 * MFM_SCHEME_MFV (reading R21): the same faces, reconstruction, face frame and wave speeds,
 * then the full HLLC flux (F_L, F_L + S_L (U*_L - U_L), F_R + S_R (U*_R - U_R)
 * or F_R by the signs of S_L, S*, S_R) in the face frame, taken back to the lab
 * frame; dm (required) receives the mass rate; no P* clamp applies.  With
 * MFM_MIXED this flux is formed in FP32 like the MFM one, dm summed in FP64.
 * limiter = 1 (reading R23): each side's reconstructed face value of each
 * field is bounded by the two centre values phi_K, phi_O (lo, hi, D = hi - lo):
 * on the side of the other particle by the midpoint interpolant + D/4, on its
 * own side by the centre range widened by D/2 (a widened bound that would
 * change sign is lo / (1 + D / (2|lo|)), likewise for hi), so positive fields
 * keep positive face states. */
mfm_status mfm_hydro_fluxes(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* solve_h + gradients + hydro_fluxes on already-ordered particles. */
mfm_status mfm_hydro_pass(mfm_ctx *ctx, mfm_particles *p, void *stream);

/* One kick-drift-kick step (reading R17) with a predicted state:
 * half kick of v and total energy with the current dp, dE; drift x with the
 * half-step velocity (wrapped on periodic axes); rebuild neighbours (which
 * REORDERS the arrays as mfm_build_neighbours does); one pass on the
 * predicted velocity and energy; second half kick; u = E/m - |v|^2/2 floored
 * at u_floor (the predicted u is floored too).  dp, dE, vsig must hold the
 * pass of the current state (mfm_hydro_pass or a previous mfm_step), and
 * hold the new state's pass on return.  dt > 0: fixed step; dt <= 0: CFL
 * step cfl * min_i H_i / vsig_i from the current vsig (reading R18), which
 * synchronises the stream.  *dt_used (nullable, host) receives the step.
 * MFM_SCHEME_MFV (reading R22): mass, momentum m v and total energy are the
 * kicked quantities, with dm, dp, dE (dm required); the half kick sets m and
 * v = (m v)/m; the pass runs on the predicted masses too; the second half
 * kick updates m, v and u in place. */
mfm_status mfm_step(mfm_ctx *ctx, mfm_particles *p, double dt, double *dt_used, void *stream);

/* Hierarchical power-of-two time steps (reading R25; the paper's section 3
 * runs particles on individual time steps): one system step of length T.
 * bins (device, int64, n, in the particles' current order; REORDERED IN PLACE
 * with them) gives each particle its bin 0 .. max_bin (max_bin <= 7); particle
 * i steps by
 * T / 2^bins[i].  A pair's level is the finer bin of its two particles and its
 * step T / 2^level.  Time advances in 2^max_bin sub-steps of T / 2^max_bin:
 * every particle drifts on each; at a sub-step boundary the levels whose step
 * divides the elapsed time are due, and only their pairs are evaluated, on the
 * state predicted with those levels' previous rates; each due level's new
 * rates close its pair step with a half kick and, before the end of T, open
 * the next one with another, applied with opposite signs to the two
 * particles of a pair (momentum and energy are conserved to rounding).
 * flags: MFM_HIER_REBIN, MFM_HIER_ACTIVE or both (other bits: MFM_E_INVALID).
 * Without MFM_HIER_ACTIVE kernel lengths and gradients are recomputed for
 * every particle at each boundary.  With it (reading R26, active subsets)
 * only the particles whose own bin is due at a boundary get new kernel
 * lengths, densities, volumes, gradient matrices and limited gradients; the
 * others keep those of their last active boundary, in nk, V, B and grad
 * (during the call B and grad hold each particle's values in the column where
 * it stood at the call's start; on return every array is in the particles'
 * current order), and enter the due pairs with their current positions and
 * predicted state.  Choosing the bins is the caller's part: with active
 * subsets, a kept particle whose flux neighbours sit several levels finer
 * keeps its geometry and coarse rates while they move, and can run away;
 * bins where flux neighbours differ by at most one level (the usual
 * neighbour time-step limiter) avoid that.
 * At the last boundary of T every level is due either way.  The per-level
 * rates live in the context (allocated on the first call, 32 doubles per
 * particle; with MFM_HIER_ACTIVE also one byte per particle and one bit per
 * cell-table entry); they are computed by a pass over the current state with
 * every level due when flags has MFM_HIER_REBIN, on the first call, when
 * max_bin changes, or after any other pass on the context.  When the
 * particles stand bit for bit where the last pass on the context left them
 * (order, positions and H, as after a hierarchical step, or after
 * mfm_hydro_pass with nothing moved since), that pass keeps the last pass's
 * kernel lengths, nk, V and gather lists and evaluates only the gradients and
 * the fluxes.  The call synchronises the stream once at its start, to check
 * on the device that every bin lies in 0 .. max_bin (else MFM_E_INVALID,
 * before anything runs) and whether the particles moved; with
 * MFM_HIER_ACTIVE also once per boundary that not every level is due, where
 * it keeps the cell tables of the last build while no particle has travelled
 * half of the finest cell since (positions may then stand just outside
 * a periodic box until the next build wraps them).  With max_bin = 0
 * the call performs mfm_step's operations for a fixed dt = T (in separate
 * kernels, equal to mfm_step's results to rounding).  MFM scheme, FP64
 * (MFM_MIXED or MFV: MFM_E_INVALID).  On return dp, dE and vsig hold the
 * rates and signal speeds of the last boundary (every level due) and the
 * counters those of its pass.  An error returned after the checks at the
 * start leaves the particles and their arrays in an unspecified state (part
 * of the system step done). */
#define MFM_HIER_REBIN 1
#define MFM_HIER_ACTIVE 2
mfm_status mfm_step_hier(mfm_ctx *ctx, mfm_particles *p, int64_t *bins, int32_t max_bin, double T, int32_t flags,
                         void *stream);

/* Copy the per-level rates that the last mfm_step_hier left (those of its last
 * boundary, every level due) into out (device, FP64, 4 x nlev x n,
 * out[(l * 4 + c) * n + i], c: dp x, y, z, dE; nlev = max_bin + 1), in the
 * current particle order.  MFM_E_STATE if there are none (no hierarchical
 * step yet, or another pass since). */
mfm_status mfm_copy_levels(mfm_ctx *ctx, double *out, void *stream);

/* The neighbour time-step limiter for the bins of mfm_step_hier (section 3's
 * individual time steps leave the choice of bins to the caller): raises each
 * bins[i] (device, int64, n, current particle order, in place) to at least
 * its flux neighbours' bins minus one, in sweeps until no bin changes, so
 * that neighbours step at most a factor 2 apart.  Uses the flux lists of the
 * last pass on these particles (MFM_E_STATE if there are none, as after
 * mfm_build_neighbours alone).  Bins outside 0 .. max_bin (max_bin <= 7):
 * MFM_E_INVALID, nothing changed.  *raised (host, nullable) receives the
 * number of raises.  Synchronises the stream once per sweep, at most
 * max_bin + 2 times. */
mfm_status mfm_limit_bins(mfm_ctx *ctx, const mfm_particles *p, int64_t *bins, int32_t max_bin, int64_t *raised,
                          void *stream);

/* Adjoint of the pass (reading R20; MFM scheme with limiter 0 only, else
 * MFM_E_INVALID): given the adjoints adj_dp (3 x n) and
 * adj_dE (n) of the pass outputs, write the adjoints of its inputs adj_x
 * (3 x n), adj_v (3 x n) and adj_u (n) = (dF/d(x, v, u))^T (adj_dp, adj_dE),
 * FP64, at fixed neighbour sets.  The kernel length enters by the
 * implicit-function theorem; limiter, Davis speeds, P* clamp and first-order
 * fallback follow the branch the forward took.  Requires that the last pass
 * on this context ran on p (its outputs nk, V, B, rho, P, grad are read).
 * All arrays are device memory in p's current order.  The first adjoint call
 * on a context allocates its adjoint scratch (120 doubles per particle). */
mfm_status mfm_hydro_pass_adjoint(mfm_ctx *ctx, const mfm_particles *p, const double *adj_dp,
                                  const double *adj_dE, double *adj_x, double *adj_v, double *adj_u,
                                  void *stream);

/* Adjoint of one fixed-dt mfm_step (reading R17/R20).  ckpt holds the state
 * at the start of the step (x, y, z, m, vx, vy, vz, u, H and its pass outputs
 * dp, dE; read only); work is a scratch particle set of the same size (every
 * array present) on which the step is recomputed.  On input the adjoint
 * arrays hold the adjoints of the state after the step (x, v, u, dp, dE) in
 * the order mfm_step leaves it; on output they hold the adjoints of the
 * checkpoint's state in the checkpoint's order.  dt must be > 0. */
mfm_status mfm_step_adjoint(mfm_ctx *ctx, const mfm_particles *ckpt, mfm_particles *work, double dt,
                            double *adj_x, double *adj_v, double *adj_u, double *adj_dp, double *adj_dE,
                            void *stream);

/* A step's tape: memory in place of recomputation for the reverse sweep
 * (reading R17/R20).  mfm_tape_bytes gives the size of one step's tape for
 * the context's capacity (about 42 doubles and 3 + max_ngb int32 per
 * particle), or -1 for a null context.
 *
 * mfm_step_taped is mfm_step with a fixed dt > 0 (MFM, per-particle limiter
 * only) that also writes into `tape` (caller-owned device memory of
 * mfm_tape_bytes bytes, overwritten) what the step's reverse reads: the state
 * after its drift and first kick, the predicted state, the pass outputs, the
 * step's permutation and its flux lists, in the order the step leaves the
 * particles.  The step itself is the same as mfm_step's, bit for bit.
 *
 * mfm_step_adjoint_taped is mfm_step_adjoint without the recomputation: it
 * reads the step from a tape written by mfm_step_taped on the state that ckpt
 * holds (ckpt: x, m, vx, vy, vz of the state at the step's start, in its
 * order; read only), and gives the same adjoints bit for bit.  The tape must
 * come from the same context parameters and particle count. */
int64_t mfm_tape_bytes(const mfm_ctx *ctx);
mfm_status mfm_step_taped(mfm_ctx *ctx, mfm_particles *p, double dt, void *tape, void *stream);
mfm_status mfm_step_adjoint_taped(mfm_ctx *ctx, const mfm_particles *ckpt, const void *tape, double dt,
                                  double *adj_x, double *adj_v, double *adj_u, double *adj_dp, double *adj_dE,
                                  void *stream);

/* Synchronise the stream of the last call and report device counters. */
mfm_status mfm_get_counters(mfm_ctx *ctx, mfm_counters *out);

/* Synchronise and turn device counters into a status: MFM_E_NOCONV,
 * MFM_E_MINIMAGE, MFM_E_CAPACITY (list overflow), MFM_E_NONFINITE, or
 * MFM_E_ILLCOND, in that order of precedence; MFM_OK otherwise. */
mfm_status mfm_check(mfm_ctx *ctx);

/* Copy the flux lists (complete once mfm_gradients has run after the last
 * mfm_solve_h; MFM_E_STATE before) into caller device buffers:
 * counts[i] (int32, n) and list[k * n + i] (int32, max_ngb x n) = index j of
 * the k-th entry of particle i, in the current particle order. */
mfm_status mfm_copy_flux_lists(mfm_ctx *ctx, int32_t *counts, int32_t *list, void *stream);

/* Flux-list slot count chosen at creation (max_ngb). */
int32_t mfm_max_ngb(const mfm_ctx *ctx);

/*
 * Kernel timing, a measurement aid outside the method itself.  While enabled,
 * every launch of the pass kernels is bracketed by a pair of HIP events
 * recorded on the call's stream: the kernel-length kernels of mfm_solve_h
 * (group scan, per-particle list solver and rescanning solver, which run back
 * to back; the counter and list resets before them are outside), the
 * gradient kernel of mfm_gradients, the flux kernel of mfm_hydro_fluxes.
 *  - mfm_set_kernel_timing(ctx, 1) enables timing and zeroes the totals;
 *    mfm_set_kernel_timing(ctx, 0) disables it.  Events are created by the
 *    library on first use and released by mfm_destroy.
 *  - mfm_kernel_time() waits for the recorded events and returns the summed
 *    duration in milliseconds and the number of timed launches of one
 *    kernel (an mfm_kernel value) since timing was last enabled.
 *  - MFM_E_INVALID for a null pointer or an unknown kernel.
 */
typedef enum { MFM_KERNEL_SOLVE_H = 0, MFM_KERNEL_GRADIENTS = 1, MFM_KERNEL_FLUXES = 2 } mfm_kernel;
mfm_status mfm_set_kernel_timing(mfm_ctx *ctx, int enable);
mfm_status mfm_kernel_time(mfm_ctx *ctx, int kernel, double *total_ms, int64_t *launches);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * pass of mfm_build_neighbours + mfm_hydro_pass without a context.
 *  - At most 8192 particles (p->n > 8192: MFM_E_CAPACITY, nothing launched),
 *    params->max_ngb <= 256 (0: 256) and params->tree_levels <= 6 (0: 6);
 *    larger values, invalid params or a missing output array: MFM_E_INVALID.
 *  - All scratch (keys, cell tables, flux lists, records, counters: about
 *    27 MB) lives in one device array inside the library, which each GPU the
 *    library runs on holds from load until the process ends.  The call makes
 *    no hipMalloc, hipFree or other allocating call on any path; counters are
 *    cleared by a kernel, not a memset.
 *  - Every call on one GPU shares that GPU's array and leaves its contents
 *    for the next call: calls that overlap on one GPU (from several streams or
 *    threads) race.
 *  - Arrays, ordering and outputs are those of the two calls it replaces: p's
 *    arrays are REORDERED IN PLACE into Morton order (id carried), then H, nk,
 *    V, B, rho, P, grad, dp, dE, vsig (and dm under MFV) are written.
 *  - counters (host, nullable): when given, the call synchronises the stream,
 *    fills it, and returns the status mfm_check would (MFM_E_NOCONV, ...); when
 *    NULL it only queues the work and never synchronises (graph capture).
 */
mfm_status mfm_hydro_pass_noalloc(const mfm_params *params, mfm_particles *p, mfm_counters *counters,
                                  void *stream);

const char *mfm_status_str(mfm_status s);
const char *mfm_last_error(const mfm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MFM_H */
