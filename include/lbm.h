/*
 * lbm.h -- C ABI of the MI355X (gfx950) solver for thermocapillary convection
 * in superimposed fluid layers: one time step of the coupled central-moment
 * lattice Boltzmann method of Elbousefi, Schupbach, Premnath and Welch,
 * "Thermocapillary convection in superimposed layers of self-rewetting
 * fluids" (arXiv 2210.07501), Secs. 3 and 4 with the moment maps of App. B.
 *
 * Problem (Sec. 1.1): a channel periodic in x, bounded by no-slip walls; the
 * bottom wall carries T_h + dT cos(2 pi x / l), the top wall T_c; fluid b
 * (phi = 1) below fluid a (phi = 0); surface tension
 * sigma(T) = sigma0 + sigma_T (T - T_ref) + sigma_TT (T - T_ref)^2
 * (Eq. ST_SRF).  Each step couples
 *   - the conservative Allen-Cahn LBM for phi (Sec. 4.1),
 *   - the pressure-based two-fluid LBM with the continuum surface force,
 *     capillary and Marangoni parts (Sec. 3 Eq. eqn6, Sec. 4.2),
 *   - the energy LBM for T (Sec. 4.3),
 * with half-way bounce-back, anti-bounce-back and free-slip walls (Sec. 5).
 *
 * Lattice conventions: node (i, j) sits at x = i, y = j (lattice units,
 * dt = dx = 1); walls are the half-way planes y = -1/2 and y = ny - 1/2; the
 * interface plane of a cold start is y = b - 1/2.  Host field arrays are
 * row-major [ny][nx] (x fastest) in float64.  Population arrays exchanged
 * with lbm_get_state / lbm_set_state are [3][9][ny][nx] float64 (f, g, h;
 * D2Q9 directions e_x = (0,1,0,-1,0,1,-1,-1,1), e_y = (0,0,1,0,-1,1,1,-1,-1)),
 * the post-streaming state of the current time level.
 *
 * Every call returns an int status (LBM_OK = 0, negative on error) except
 * lbm_destroy and lbm_strerror.  A context is used by one host thread at a
 * time.  All work, set-up copies included, is ordered on the context's HIP
 * stream.  lbm_step only enqueues; every other call that touches the device
 * synchronises that stream (never the whole device) before it returns.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameters                   */
    LBM_ENOMEM = -2,     /* device allocation failed                          */
    LBM_EDEVICE = -3,    /* HIP runtime error (text kept for lbm_strerror)    */
    LBM_EDIVERGED = -4,  /* non-finite value found by the residual reduction  */
    LBM_ESTATE = -5      /* call out of order (e.g. step before init)         */
};

typedef enum {
    LBM_FP64 = 0,        /* populations stored and collided in float64        */
    LBM_FP32_DEV = 1     /* populations stored in float32 as deviations from
                            reference equilibria; the phase-field and the
                            hydrodynamic collisions, the residual and the
                            conserved sums are float64                        */
} lbm_precision;

/* Parameters of one channel (lattice units; rho c_p = 1 for both fluids). */
typedef struct {
    int32_t nx, ny;      /* lattice size; nx >= 4, ny >= 4                    */
    int32_t n_waves;     /* heating wavelengths along x, l = nx / n_waves     */
    int32_t reserved;    /* must be 0                                         */
    double b;            /* bottom-layer thickness (cold-start interface plane
                            at y = b - 1/2), W < b < ny - W                   */
    double W, M_phi;     /* interface width and Allen-Cahn mobility (Sec. 3)  */
    double rho_a, rho_b; /* densities: a = top (phi = 0), b = bottom (phi = 1) */
    double mu_a, mu_b;   /* dynamic viscosities (Eq. eqn11, linear in phi)    */
    double k_a, k_b;     /* thermal conductivities (linear in phi)            */
    double sigma0, sigma_T, sigma_TT, T_ref;  /* Eq. (ST_SRF)                  */
    double T_h, dT, T_c; /* walls: T_h + dT cos(2 pi x / l) bottom, T_c top   */
    double Fx_ext, Fy_ext; /* external body force density (Sec. 3, Eq. eqn5)  */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Device allocator hooks (for example a framework's caching allocator).
 * alloc returns a device pointer of at least `bytes` bytes, 256-byte aligned,
 * or NULL; free releases it.  Both NULL: the library uses hipMalloc/hipFree. */
typedef void* (*lbm_alloc_fn)(size_t bytes, void* user);
typedef void (*lbm_free_fn)(void* ptr, void* user);

/* Create a context for n_inst independent channels (params[0..n_inst-1])
 * that are stepped together by single launches.  precision: lbm_precision.
 * hip_stream: the hipStream_t to order all work on (NULL: the null stream).  Rejects (LBM_EINVAL): n_inst <= 0,
 * nx or ny < 4, nx * ny above 19 884 107 nodes (27 x 8 x nx x ny must stay below
 * 2^32), n_waves <= 0 or not dividing nx, W <= 0, b outside
 * (W, ny - W), non-positive densities, viscosities, conductivities or
 * mobility.  On success *out owns all device memory of the context. */
int lbm_create(const lbm_params* params, int32_t n_inst, int32_t precision, void* hip_stream,
               lbm_alloc_fn alloc, lbm_free_fn free_fn, void* user, lbm_ctx** out);

/* Initialise every instance at equilibrium (no sharpening flux) from fields.
 * fields == NULL: cold start -- fluid at rest, p = 1/3, phi a tanh profile
 * of width W centred on y = b - 1/2, T linear between the two walls in each
 * column.  Otherwise fields holds, for each instance in order, the host
 * arrays phi, ux, uy, T ([ny][nx] each, concatenated).  Resets step counts
 * and residual history. */
int lbm_init(lbm_ctx* ctx, const double* fields);

/* As lbm_init from given fields, but fields is device memory in the same
 * layout (for each instance in order: phi, ux, uy, T, [ny][nx] each) -- the
 * hand-off from a field predictor such as the warm-start network
 * (nn_to_fields writes this layout).  The values are not checked on the
 * host: a non-finite value shows up as LBM_EDIVERGED at the first check.
 * LBM_EINVAL if fields is NULL. */
int lbm_init_device(lbm_ctx* ctx, const double* fields);

/* Advance every active instance by n >= 0 time steps (stream-ordered, no
 * synchronisation).  Every 100th step (counted from init) also records the
 * float64 residual, sum phi, sum rho and the peak interface velocity. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Step all instances until each one's residual is <= r_tol (then it stops
 * advancing) or max_steps steps have been taken.  Replays a captured HIP
 * graph of 100 steps; synchronises.  *n_active (may be NULL) receives the
 * number of instances still above r_tol.  Returns LBM_EDIVERGED if any
 * instance produced a non-finite value. */
int lbm_solve(lbm_ctx* ctx, double r_tol, int64_t max_steps, int32_t* n_active);

/* Macroscopic fields of instance inst at the current time level (the
 * corrected u and p of Sec. 4.2).  Caller-owned host arrays [ny][nx]; any
 * pointer may be NULL.  Synchronises. */
int lbm_fields(lbm_ctx* ctx, int32_t inst, double* phi, double* ux, double* uy, double* T,
               double* p);

/* Last recorded check of instance inst: residual r (+inf before two checks),
 * sum phi, sum rho(phi), peak |u_x| on the phi = 1/2 level, steps advanced.
 * Any pointer may be NULL.  Synchronises.  Returns LBM_EDIVERGED if the
 * check saw a non-finite value. */
int lbm_residual(lbm_ctx* ctx, int32_t inst, double* r, double* sum_phi, double* sum_mass,
                 double* u_int_peak, int64_t* steps_done);

/* Retire instance inst now, as if it had converged at the current step:
 * later steps and solves leave it untouched, and lbm_residual reports its
 * last check.  Its state stays readable (and writable through
 * lbm_set_state).  No effect on a retired instance.  LBM_ESTATE before
 * the first step after init.  Synchronises. */
int lbm_retire(lbm_ctx* ctx, int32_t inst);

/* Start instance inst again from fields, at any step, leaving the other
 * instances untouched: its populations are set to the equilibrium of the
 * fields exactly as lbm_init sets them (fields NULL: the cold start from
 * rest), its residual history and retirement are cleared and it takes part
 * in later steps and solves again.  fields: host arrays phi, ux, uy, T of
 * this instance ([ny][nx] each, concatenated).  The instance's reported step
 * count keeps counting from the context's steps (so a restart after a
 * divergence is charged the steps already spent).  This is the fallback of
 * a warm-started solve: a channel whose start diverged (LBM_EDIVERGED) is
 * restarted from rest.  LBM_EINVAL for a bad index or a non-finite field
 * value, LBM_ESTATE before lbm_init.  Synchronises. */
int lbm_restart(lbm_ctx* ctx, int32_t inst, const double* fields);

/* Raw populations of instance inst, float64 [3][9][ny][nx] (host).  Syncs. */
int lbm_get_state(lbm_ctx* ctx, int32_t inst, double* pop);
/* Overwrite instance inst with populations (host, float64 [3][9][ny][nx]). */
int lbm_set_state(lbm_ctx* ctx, int32_t inst, const double* pop);

/* Time n back-to-back launches of the fused step kernel alone with HIP
 * events on the context stream; *ms receives the average per launch.
 * Advances the state by n steps without the residual checks (the next check
 * reports its own step index).  Synchronises. */
int lbm_profile_steps(lbm_ctx* ctx, int64_t n, double* ms);

/* Tile shape of the fused step kernel: tx x ty nodes per workgroup from the
 * compiled set {64x8 (default), 32x8, 64x4, 16x16, 64x16, 128x8}; 0,0 picks
 * the default.  LBM_EINVAL for any other shape. */
int lbm_set_tile(lbm_ctx* ctx, int32_t tx, int32_t ty);

/* Autotuner: time `reps` launches of the fused step kernel for every
 * compiled tile shape on this context's channels and keep the fastest.  The
 * state is not advanced (each launch gathers from the current buffer and
 * writes the other one).  Outputs (may be NULL): chosen shape and its time
 * per launch in ms.  Synchronises. */
int lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* tx, int32_t* ty, double* ms);

/* Number of lattice nodes over all instances, and the device bytes the
 * context holds: every live allocation (through the caller's allocator when
 * one was given), rounded up to 256 bytes each. */
int lbm_info(lbm_ctx* ctx, int64_t* nodes, int64_t* device_bytes);

void lbm_destroy(lbm_ctx* ctx);
const char* lbm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
