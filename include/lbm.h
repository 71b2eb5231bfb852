/*
 * lbm.h - C ABI of the MI355X (gfx950) phase-change lattice-Boltzmann step.
 *
 * The method is the three-population BGK scheme of Verdier, Kestener and
 * Cartalade (arXiv 2003.06342): a conservative Allen-Cahn phase field phi
 * with interface mass production (Sec. 2.1, Eqs. CAC_ChgtPhase and
 * ProductionRate; LB scheme Sec. 3.2), incompressible Navier-Stokes with
 * surface tension mu*grad(phi) and buoyancy (Eqs. ConservMasse_ChgtPhase,
 * ConvservQDM_ChgtPhase, Force_Total, ChemicalPotential; LB scheme Sec.
 * 3.1) and the heat equation with latent heat (Eq. Temperature_ChgtPhase;
 * LB scheme Sec. 3.3), coupled by the isotropic gradient and Laplacian of
 * Sec. 3.4.  All quantities are in lattice units (dx = dt = 1).
 *
 * Conventions
 *   - Field arrays are C-ordered [nz][ny][nx] (nz = 1 in 2-D), x fastest.
 *     Node (i, j, k) has its centre at (i+1/2, j+1/2, k+1/2); a wall axis
 *     has half-way walls on the planes 0 and n.
 *   - Every pointer argument named dev_* or documented as "device" is a HIP
 *     device pointer on the context's device.  Host pointers are marked.
 *   - Ownership: the caller owns every buffer.  The library never allocates
 *     device memory: it borrows the workspace given to lbm_create for the
 *     lifetime of the context and field/state pointers for the duration of
 *     one call.  The context object itself is host memory owned by the
 *     library (freed by lbm_destroy).
 *   - Calls are asynchronous and ordered on the stream given to lbm_create
 *     unless documented as synchronising.  A context must not be used from
 *     two threads at once.
 *   - Errors: every call returns an lbm_status; nothing throws across the
 *     ABI.  lbm_last_error() gives a message for the last failure on the
 *     calling thread.  Faults of earlier asynchronous work surface as
 *     LBM_E_HIP at the next synchronising call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef int32_t lbm_status;

#define LBM_OK 0
#define LBM_E_INVAL (-1)        /* invalid argument or parameter set        */
#define LBM_E_NOMEM (-2)        /* a caller buffer is too small             */
#define LBM_E_HIP (-3)          /* the HIP runtime reported an error        */
#define LBM_E_STATE (-4)        /* call made in the wrong order             */
#define LBM_E_UNSTABLE (-5)     /* non-finite values in the diagnostics     */
#define LBM_E_UNSUPPORTED (-6)  /* valid but not built (lattice/BC combo)   */

/* Lattices (Sec. 3): D2Q9 in 2-D for f, g and s; in 3-D D3Q19 for f and
 * D3Q7 for g and s.  Stencils use D2Q9 in 2-D and D3Q19 in 3-D.  D2Q5
 * (w = 1/2, 1/8; c_s^2 = 1/4), the z-projection of D3Q7, may carry g and s
 * in 2-D (both): a z-invariant 3-D run then equals the 2-D run. */
enum { LBM_D2Q9 = 9, LBM_D2Q5 = 5, LBM_D3Q7 = 7, LBM_D3Q19 = 19 };

/* Population storage.  F16_DEV / BF16_DEV store each population as the
 * 16-bit float (value - w_i * ref) * 2^k with a power-of-two scale;
 * arithmetic is FP32.  ref is a constant for f; for the phase-field family g
 * it is the lagged phi of the node that reads the population; for the
 * temperature family s it is T_ref(x), the temperature of the node x that
 * stored the population, kept as one more FP32 plane of the state.  Lagged
 * scalars stay FP32. */
enum { LBM_ST_F64 = 0, LBM_ST_F32 = 1, LBM_ST_F16_DEV = 2, LBM_ST_BF16_DEV = 3 };

/* Per-axis boundary: periodic, or half-way walls on both faces.  A wall is
 * a no-slip bounce-back wall for f (Sec. 4.1.2) and an anti-bounce-back
 * Dirichlet wall for g and s (Sec. 3.3) with the face values phi_wall and
 * T_wall (T_wall may be set per node with lbm_set_wall_T). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1 };

/* Model switches. */
enum {
  LBM_NS = 1,            /* evolve f (else u = 0, p = 0)                    */
  LBM_HEAT = 2,          /* evolve s (else T = 0 and no phase change)       */
  LBM_PHASE_CHANGE = 4,  /* production q = m'''/rho_g of Eq. ProductionRate */
  LBM_VISC_LINEAR = 8,   /* Eq. Visco_lin instead of the harmonic Eq. Viscosity */
  LBM_GEQ_CAC = 16,      /* CAC equilibrium form of Eq. Geq_AC-1            */
  LBM_DIV_LOCAL = 32     /* div(u phi) of the latent-heat source taken as
                          * u.grad(phi) + phi m''' (1/rho_g - 1/rho_l), from
                          * div(u) of Eq. ConservMasse_ChgtPhase, with the
                          * production of the previous step (radius-1 form);
                          * default: the central stencil of Eq. Grad applied
                          * to u_a phi (radius 2)                            */
};

/* Collision operator of all three families (Sec. 3, the remark after Eq.
 * LBE: TRT and MRT reach lower mobility and higher Peclet numbers than BGK).
 *   BGK: one rate per family, omega = 1/(tau + 1/2), tau = diffusivity/c_s^2.
 *   TRT: the parts of (pop - eq + S/2) symmetric and antisymmetric under
 *        c -> -c relax with omega+ and omega-.  The rate of the transport
 *        coefficient is the BGK rate (omega+ for f: viscosity; omega- for g
 *        and s: mobility, diffusivity); the other follows from the magic
 *        parameter Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) (trt_lambda).
 *   MRT: (pop - eq + S/2) is relaxed in an orthogonal moment basis (D2Q9:
 *        rho, e, eps, jx, qx, jy, qy, pxx, pxy; D3Q7: 1, cx, cy, cz,
 *        7c^2 - 6, 2cx^2 - cy^2 - cz^2, cy^2 - cz^2).  The transport moments
 *        relax at the BGK rate (pxx, pxy for f; jx, jy(, jz) for g and s);
 *        the others at mrt_rates[family] = {s_e, s_eps, s_q, s_p}: the
 *        zeroth moment at s_e, j of f at s_q, pxx/pxy of g and s (and the two
 *        D3Q7 second-order moments) at s_p.  Not built for D3Q19. */
enum { LBM_COLL_BGK = 0, LBM_COLL_TRT = 1, LBM_COLL_MRT = 2 };

/* Directional derivative c_i . grad(phi) in the NS source (Eq. Forcing:
 * c_i . grad(rho) and the surface tension mu c_i . grad(phi)): the
 * projection of the central Eq. Grad vector, or the first- or second-order
 * biased (upwind) differences along c_i that Sec. 3.4 lists after Eq.
 * Laplacian, phi(x + c_i) - phi(x) and [-phi(x + 2c_i) + 4 phi(x + c_i) -
 * 3 phi(x)] / 2.  Every vector use of grad(phi) (velocity, pressure, the
 * normal of the phase-field source, whose zeroth moment must vanish for phi
 * to stay conserved) and the Laplacian keep the central stencils.  Ghosts
 * two nodes beyond a wall mirror the second node from it. */
enum { LBM_GRAD_CENTRAL = 0, LBM_GRAD_BIASED1 = 1, LBM_GRAD_BIASED2 = 2 };

/* dtype of caller field arrays */
enum { LBM_DT_F32 = 0, LBM_DT_F64 = 1 };

/* Field selection bits of lbm_get_fields; output planes follow bit order. */
enum {
  LBM_FIELD_PHI = 1, LBM_FIELD_P = 2, LBM_FIELD_UX = 4, LBM_FIELD_UY = 8,
  LBM_FIELD_UZ = 16, LBM_FIELD_T = 32
};

typedef struct {
  int32_t dim;                   /* 2 or 3                                     */
  int32_t nx, ny, nz;            /* nodes per axis, nz = 1 in 2-D              */
  int32_t lat_f, lat_g, lat_s;   /* LBM_D2Q9 (2-D) or LBM_D3Q19/LBM_D3Q7 (3-D) */
  int32_t storage;               /* LBM_ST_*                                   */
  uint32_t flags;                /* LBM_NS | LBM_HEAT | ...                    */
  /* transport: nu = tau_f c_s^2, M = tau_g c_s^2, alpha = tau_s c_s^2
   * (Sec. 3.1-3.3); liquid is phi = 0, vapour phi = 1                      */
  double nu_l, nu_g, mobility, alpha_l, alpha_g;
  /* interface width W, surface tension sigma (Eq. Def_K-H), densities      */
  double W, sigma, rho_l, rho_g;
  /* L/Cp, saturation temperature, interface temperature theta_I and the
   * coefficient A of Eq. ProductionRate (0 selects 10/48, App. B)           */
  double L_over_cp, T_sat, theta_I, A_coef;
  double gravity[3];             /* acceleration vector; buoyancy (rho - rho_l) g */
  double body_force[3];          /* uniform force density added to F_tot     */
  int32_t bc[3];                 /* LBM_BC_* per axis x, y, z                 */
  double phi_wall[3][2];         /* [axis][lo, hi] anti-bounce-back phi       */
  double T_wall[3][2];           /* [axis][lo, hi] anti-bounce-back T         */
  double eps_n;                  /* n = grad phi / sqrt(|grad phi|^2 + eps_n^2) (0 -> 1e-3) */
  int32_t collision;             /* LBM_COLL_*                                 */
  double trt_lambda[3];          /* TRT magic parameter of f, g, s (0 -> 1/4)  */
  double mrt_rates[3][4];        /* MRT free rates of f, g, s: s_e, s_eps, s_q, s_p, each in (0, 2) */
  int32_t grad_scheme;           /* LBM_GRAD_*                                 */
  int32_t check_every;           /* > 0: lbm_step checks the fields for non-finite
                                  * values every check_every steps (FP64
                                  * reduction; synchronises) and returns
                                  * LBM_E_UNSTABLE at the first failure     */
  /* Per wall face [axis][lo, hi], the condition of f: LBM_FBC_NOSLIP
   * (half-way bounce-back, Sec. 4.1.2) or LBM_FBC_PRESSURE, an open face at
   * pressure p_wall: the pressure anti-bounce-back f_i = -f_{i'} + 2 w_i
   * p_wall (the even part of Eq. Feq_NS_Incompr at the face pressure, its
   * O(u^2) terms dropped) with a zero-gradient velocity ghost for the
   * stencils.  g and s keep their Dirichlet anti-bounce-back.  Lets the
   * vapour produced by evaporation leave a closed box, whose gauge pressure
   * otherwise drifts.  Only on walled axes (LBM_E_INVAL otherwise). */
  int32_t f_bc[3][2];
  double p_wall[3][2];
} lbm_params;
enum { LBM_FBC_NOSLIP = 0, LBM_FBC_PRESSURE = 1 };
/* Kernels: BGK with central derivatives and the radius-2 div(u phi) runs the
 * default step kernels; any of TRT / MRT, a biased scheme or LBM_DIV_LOCAL
 * (which needs LBM_NS | LBM_HEAT) runs the extended step kernels, with the
 * same memory traffic. */

/* Bytes of device workspace lbm_create needs for these parameters
 * (populations A and B, lagged phi and q, wall rows, reduction scratch).
 * Returns LBM_E_INVAL / LBM_E_UNSUPPORTED for parameter sets that
 * lbm_create would reject. */
lbm_status lbm_workspace_size(const lbm_params* prm, size_t* bytes);

/* Validate the parameters (tau > 0, omega = 1/(tau + 1/2) < 2 for the
 * extreme phases, rho > 0, W > 0, lattice/dimension pairs, at least 2 nodes
 * along a walled axis) and build a
 * context that uses `dev_workspace` (>= lbm_workspace_size bytes, 256-byte
 * aligned, owned by the caller) and launches on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  *out is NULL on failure. */
lbm_status lbm_create(const lbm_params* prm, void* dev_workspace, size_t bytes,
                      void* hip_stream, lbm_ctx** out);

/* Initialise the populations from phi0, T0 (device arrays [nz][ny][nx]) and
 * the optional u0 ([3][nz][ny][nx], NULL = 0) and p0 (NULL = 0): every
 * population is set to its equilibrium minus half its source at these
 * fields, so that the moments of the first step return them exactly.
 * T0 is ignored without LBM_HEAT.  dtype = LBM_DT_F32 or LBM_DT_F64.
 * Discards a recorded adjoint tape. */
lbm_status lbm_init_fields(lbm_ctx* ctx, const void* phi0, const void* T0,
                           const void* u0, const void* p0, int32_t dtype);

/* Per-node wall temperature on face (axis, side): a device array over the
 * other two axes in [..][..] C order (2-D y wall: nx values; 3-D z wall:
 * [ny][nx]).  Takes effect for the following steps; discards a recorded
 * adjoint tape (its recomputation would use the new wall values). */
lbm_status lbm_set_wall_T(lbm_ctx* ctx, int32_t axis, int32_t side,
                          const void* dev_face, int32_t dtype);

/* Advance nsteps time steps (asynchronous, stream-ordered).  Each step is
 * one fused pass: pull streaming with wall links, moments, stencils,
 * closures, equilibria, sources and collision of f, g and s.  With
 * check_every > 0 the call synchronises every check_every steps and returns
 * LBM_E_UNSTABLE (after the step that produced them) if any node's phi, T,
 * u or p is non-finite; lbm_get_step then tells how far it got. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Write the macroscopic fields selected by `mask` (LBM_FIELD_* bits) at the
 * current populations into dev_out, one [nz][ny][nx] plane per selected
 * field in bit order, as dtype.  phi, u, p, T follow Eqs. Moment_Phi,
 * Velocity, Pressure and Moment_Temp. */
lbm_status lbm_get_fields(lbm_ctx* ctx, uint32_t mask, void* dev_out, int32_t dtype);

/* FP64 diagnostics at the current populations (host out[5]): sum(phi),
 * enthalpy sum(T) + (L/Cp)(sum(phi) + sum(phi_prev))/2, vapour fraction
 * sum(phi)/N, max|u|, and the count of non-finite nodes.  Deterministic
 * (fixed reduction tree).  Synchronises the stream; returns
 * LBM_E_UNSTABLE if the count is non-zero. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, double out[5]);

/* Checkpoint / resume: the raw state (populations, lagged phi and q, and
 * T_ref for 16-bit storage) as an opaque byte blob of lbm_state_size bytes,
 * copied device-to-device.  lbm_set_state discards a recorded adjoint tape
 * and resets the step count to 0. */
lbm_status lbm_state_size(const lbm_ctx* ctx, size_t* bytes);
lbm_status lbm_get_state(lbm_ctx* ctx, void* dev_out, size_t bytes);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* dev_in, size_t bytes);

/* Steps taken since lbm_init_fields / lbm_set_state (host out). */
lbm_status lbm_get_step(const lbm_ctx* ctx, int64_t* out);

/* Wait for all work queued on the context's stream; reports HIP errors. */
lbm_status lbm_sync(lbm_ctx* ctx);

/* ---- Adjoint (2-D, FP32 or FP64 storage, LBM_NS | LBM_HEAT, BGK collision,
 * central gradients, at most one walled axis).  Gradients of a loss
 * L(phi^N, T^N) of the final phase field and temperature with respect to
 * the initial phase field phi0, the initial temperature T0 and a
 * wall-temperature row, by a hand-written reverse sweep of the fused step
 * (transposed node Jacobian, transposed stencils, transposed pull gather;
 * the anti-bounce-back links of Sec. 3.3 carry T_w linearly). */

/* Checkpointing policy of the tape.  SQRT: snapshots every K = ceil(sqrt(N))
 * steps plus one recomputed segment of K states (memory O(sqrt N) states,
 * N - ceil(N/K) recomputed steps).  BINOMIAL: binomial checkpointing
 * (Griewank and Walther): s checkpoints, the fewest with C(s + 3, 3) >= N,
 * plus two work states, so that no step is recomputed more than three
 * times (N = 2000: 23 states against 90, about 1.9 N recomputed steps
 * against 0.98 N).  Both give the same gradients bit for bit. */
enum { LBM_TAPE_SQRT = 0, LBM_TAPE_BINOMIAL = 1 };

/* Bytes of the tape for nsteps under `policy`. */
lbm_status lbm_tape_size(const lbm_ctx* ctx, int64_t nsteps, int32_t policy, size_t* bytes);

/* Advance nsteps from a freshly initialised state while recording the tape
 * in dev_tape (caller-owned, 256-byte aligned, >= lbm_tape_size bytes;
 * borrowed until the next lbm_forward_taped).  The context must be at step
 * 0 of an lbm_init_fields call with u0 == NULL (the reverse sweep
 * differentiates that initialisation): otherwise LBM_E_STATE.
 * Asynchronous. */
lbm_status lbm_forward_taped(lbm_ctx* ctx, int64_t nsteps, int32_t policy, void* dev_tape,
                             size_t bytes);

/* Bytes of the scratch workspace lbm_backward needs. */
lbm_status lbm_adjoint_workspace_size(const lbm_ctx* ctx, size_t* bytes);

/* Reverse sweep over the taped steps.  Seeds (device arrays [ny][nx] of
 * seed_dtype, each nullable, at least one given): g_phi = dL/dphi^N and
 * g_T = dL/dT^N at the fields lbm_get_fields returns after the taped run.
 * g_u and g_p (dL/du^N, dL/dp^N) must be NULL: LBM_E_UNSUPPORTED otherwise.
 * dev_ws: >= lbm_adjoint_workspace_size bytes, 256-byte aligned.  Writes
 * (each nullable) d_phi0 [ny][nx], d_T0 [ny][nx] and the gradient of the
 * wall-temperature face (tw_axis, tw_side) (nx values for a y wall) as
 * out_dtype.  The context's current state is left at step N.  Returns
 * LBM_E_STATE without a tape, or if the context stepped, was
 * re-initialised, had its state set or a wall temperature changed after
 * lbm_forward_taped.  Asynchronous. */
lbm_status lbm_backward(lbm_ctx* ctx, const void* g_phi, const void* g_T, const void* g_u,
                        const void* g_p, int32_t seed_dtype, void* dev_ws, size_t ws_bytes,
                        void* d_phi0, void* d_T0, void* d_Twall, int32_t tw_axis,
                        int32_t tw_side, int32_t out_dtype);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lbm_backward with its scratch workspace taken from a static device array
 * of the library instead of dev_ws.  The array holds
 * LBM_STATIC_SCRATCH_BYTES on every device the library runs on, from module
 * load until the process ends; the adjoint workspace of a 512 x 512 FP32
 * film (70 MiB) fits.  Arguments, seeds, outputs, errors and the tape are
 * those of lbm_backward; returns LBM_E_NOMEM when
 * lbm_adjoint_workspace_size exceeds the array.  Allocates nothing.  Every
 * call on one GPU shares that GPU's array and leaves it holding its
 * intermediates (each call clears what must start at zero): calls that
 * overlap in time on one GPU race, so serialise them (one stream, or an
 * event between them).  Asynchronous. */
#define LBM_STATIC_SCRATCH_BYTES (128u << 20)
lbm_status lbm_backward_static(lbm_ctx* ctx, const void* g_phi, const void* g_T, const void* g_u,
                               const void* g_p, int32_t seed_dtype, void* d_phi0, void* d_T0,
                               void* d_Twall, int32_t tw_axis, int32_t tw_side, int32_t out_dtype);

void lbm_destroy(lbm_ctx* ctx);

/* Message of the last error on the calling thread (never NULL). */
const char* lbm_last_error(void);

/* Library version string. */
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
