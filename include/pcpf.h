/*
 * pcpf.h -- C ABI of the MI355X (gfx950) FR-PCPF library.
 *
 * The library evaluates the Flux Reconstruction (FR) residual of the preconditioned,
 * localized conservative phase-field system of Al-Salami, Kamra & Hu (arXiv 2006.10967)
 * on affine quadrilateral / hexahedral tensor-product elements and advances it with the
 * classic four-stage Runge-Kutta scheme on one GPU:
 *
 *   u = [phi, psi],  du/dt + div f(u, grad u) = 0                      (§3.1)
 *   f = [phi v - max(gamma,|v|) (eps grad phi - gamma phi (1-phi) n); psi v],
 *   n = grad psi / |grad psi|                                          (§2)
 *   psi reset to phi - 1/2 every N steps, then preconditioned by pseudo-time iterations of
 *   dpsi/dtau = div(nu_s grad psi) + sgn(psi0) (1 - |grad psi|)         (§2, §3.2)
 *
 * Conventions
 *   - All functions return pcpf_status; no C++ exception crosses the ABI.
 *   - "host" pointers point to CPU memory, "d_" pointers to device memory of the GPU that is
 *     current when pcpf_create is called. Host arrays are copied; the caller may free them
 *     when the call returns.
 *   - Work is enqueued on the HIP stream given to pcpf_create (borrowed, not owned) and is
 *     asynchronous unless stated otherwise.
 *   - One context may not be used from two threads at once. Identical inputs give bitwise
 *     identical outputs (no floating-point atomics).
 *   - Element e, solution point i: i = sum_k i_k n^k over the n = p+1 Gauss-Legendre
 *     points per direction (i_0 fastest). A per-point field is an array [E][N_u],
 *     N_u = n^d, in the state type of the context (double for PCPF_FP64, float for
 *     PCPF_FP32 and PCPF_BF16).
 *   - Face f = 2k + s of an element is the face at reference coordinate xi_k = -1 (s = 0)
 *     or +1 (s = 1). Face 2k+1 of element e must meet face 2k of nbr[e][2k+1] with the
 *     tangential reference axes of both faces pointing the same way in space.
 */
#ifndef PCPF_H
#define PCPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCPF_ABI_VERSION 2
#define PCPF_MAX_ORDER 6

typedef enum pcpf_status {
    PCPF_OK = 0,
    PCPF_EINVAL = 1,        /* invalid argument: sizes, pointers, parameters, connectivity */
    PCPF_EDEVICE = 2,       /* a HIP runtime call failed; pcpf_last_error has its message */
    PCPF_EUNSUPPORTED = 3,  /* valid but not built (e.g. order above the compiled range) */
    PCPF_ESTATE = 4,        /* call out of order (no state set, ...) */
    PCPF_ENONFINITE = 5,    /* the state became non-finite or |phi| > 10; state kept */
    PCPF_ENOMEM = 6         /* a host allocation failed (the library caught the exception) */
} pcpf_status;

/* Precision of the form. PCPF_FP64: everything in float64. PCPF_FP32: float32 state and
 * arithmetic. PCPF_BF16: float32 state and pointwise arithmetic, with the element line
 * operators of the gradient and the divergence (§3.1 Steps 3 and 6) applied on the matrix
 * cores with bfloat16 operands and float32 accumulation. Reductions and the LOGIT reset
 * are float64 in every form. */
enum { PCPF_FP64 = 0, PCPF_FP32 = 1, PCPF_BF16 = 2 };
enum { PCPF_VEL_UNIFORM = 0, PCPF_VEL_ROTATION = 1,           /* analytic velocity kinds */
       PCPF_VEL_SINGLE_VORTEX = 2, PCPF_VEL_LEVEQUE3D = 3 };
enum { PCPF_RESET_LINEAR = 0, PCPF_RESET_LOGIT = 1 };         /* psi reset transform */
enum { PCPF_MODE_PHYS = 0, PCPF_MODE_PRECOND = 1 };           /* residual kind */
enum { PCPF_REDUCE_MASS = 0, PCPF_REDUCE_L1 = 1,              /* FP64 reductions */
       PCPF_REDUCE_RMS = 2 };
enum { PCPF_NORMAL_PSI = 0,  /* interface normal grad psi / |grad psi| (§2, the method) */
       PCPF_NORMAL_PHI = 1 };/* grad phi / |grad phi|: the unpreconditioned conservative phase
                                field of §2 (psi is still advected but not used) */
/* Smeared sign of the preconditioning equation (§2, Eq. lsequation and the text after it:
 * tanh(psi0 / |grad psi|)). */
enum { PCPF_SGN_PSI0 = 0,    /* |grad psi0| of the reset, once per reset (default; equals
                                the printed form at the first pseudo stage) */
       PCPF_SGN_CURRENT = 1 };/* |grad psi| of the current pseudo stage (the printed form) */
/* Stop rule of the pseudo-time iterations (§3.2, after Eq. pseudotimesystem). */
enum { PCPF_STOP_FIXED = 0,  /* exactly precond_iters iterations (default) */
       PCPF_STOP_RMS = 1 };  /* stop after the first iteration k with
                                sqrt(mean over all E N_u points of ((psi^k - psi^(k-1))/dtau)^2)
                                <= 1/2, at most precond_iters iterations */

/* Mesh and FR operators (host memory, float64, row-major). */
typedef struct pcpf_mesh {
    int32_t ndims;           /* d: 2 (quads) or 3 (hexes) */
    int32_t order;           /* p: 1..PCPF_MAX_ORDER (3D: 1..5); n = p + 1 */
    int64_t nelem;           /* E >= 1 */
    /* 1D factors of the tensor-product element (§3.1, Steps 1, 3 and 6) */
    const double* nodes;     /* [n]   solution points xi_a on [-1, 1], ascending */
    const double* weights;   /* [n]   quadrature weights w_a of the nodes */
    const double* deriv;     /* [n*n] deriv[a*n + b] = l_b'(xi_a) (nodal derivative) */
    const double* lminus;    /* [n]   l_a(-1): interpolation to the xi = -1 end */
    const double* lplus;     /* [n]   l_a(+1): interpolation to the xi = +1 end */
    const double* cminus;    /* [n]   divergence of the correction function of the
                                      xi = -1 end at node a (DG: l_a(-1)/w_a) */
    const double* cplus;     /* [n]   same for the xi = +1 end (DG: l_a(+1)/w_a) */
    const double* vinv;      /* [n*n] vinv[j*n + a]: coefficient j of the orthonormal
                                      Legendre expansion from nodal values (sensor, §3.2) */
    /* affine geometry: x = x0 + J (xi + 1) */
    const double* x0;        /* [E*d]   image of the reference corner (-1, ..., -1) */
    const double* jac;       /* [E*d*d] J[i][j] = dx_i / dxi_j, det J > 0 */
    const int32_t* nbr;      /* [E*2d]  element across face f, -1 = boundary (ghost state
                                        equal to the interior state, §3.3) */
    double period[3];        /* domain period along each physical axis (0 = not periodic):
                                paired face points must coincide up to a translation by
                                integer multiples of these periods */
} pcpf_mesh;

/* Method parameters (§2, §3.2, §4). */
typedef struct pcpf_params {
    double gamma;        /* sharpening weight and floor of |v| in max(gamma, |v|) (0.09) */
    double eps;          /* interface diffusion eps (0.06 h / p) */
    double eps_w;        /* width of the tanh kernel, used by the LOGIT reset */
    double tau;          /* LDG jump penalty, dissipative sign (0.1) */
    double nu_max;       /* maximum artificial viscosity (0.15 h / p) */
    double s0;           /* sensor threshold (-5) */
    double kappa;        /* sensor ramp half width (5) */
    double dtau;         /* pseudo-time step of the preconditioning iterations */
    double delta_n;      /* |grad psi| regularisation of the normal (1e-12) */
    double delta_g;      /* floor of |grad psi0| in the smeared sign (1e-12) */
    double delta_phi;    /* clamp of phi in the LOGIT reset (1e-12) */
    double vel_amp;      /* velocity amplitude A: v = A v0(x) g(t) */
    double vel_period;   /* T in g(t) = cos(pi t / T) (vortex and LeVeque kinds) */
    double vel_u0[3];    /* PCPF_VEL_UNIFORM: the constant velocity; PCPF_VEL_ROTATION: the
                            centre (u0[0], u0[1]) of the rotation (c_y - y, x - c_x) */
    int32_t vel_kind;    /* PCPF_VEL_* */
    int32_t reset_mode;  /* PCPF_RESET_* */
    int32_t reset_every; /* reset + precondition before steps with index % N == 0 (0: never) */
    int32_t precond_iters; /* pseudo-time RK4 iterations per reset (>= 0); the cap of
                              PCPF_STOP_RMS */
    int32_t precision;   /* PCPF_FP64, PCPF_FP32 or PCPF_BF16 */
    int32_t normal_mode; /* PCPF_NORMAL_PSI (default) or PCPF_NORMAL_PHI */
    int32_t sgn_mode;    /* PCPF_SGN_PSI0 (default) or PCPF_SGN_CURRENT */
    int32_t stop_mode;   /* PCPF_STOP_FIXED (default) or PCPF_STOP_RMS */
} pcpf_params;

/* Element shapes of a dense description. */
enum { PCPF_SHAPE_TENSOR = 0,   /* quadrilateral (d = 2) / hexahedral (d = 3) element */
       PCPF_SHAPE_TRIANGLE = 1 };/* triangle (d = 2) */

/* The mesh and FR operators in the dense form the method is written in (§3.1, Steps 1-6:
 * each operator an N_f x N_u or N_u x N_u matrix acting on the values of one element), the
 * per-element affine geometry (§3.1 mapping, Jacobian and transformed-flux equations) and
 * the per-flux-point connectivity (§3.1 Step 2: each flux point of a face paired with
 * the coincident flux point of the neighbouring element). Host memory, row-major, float64
 * unless stated. Tensor elements: solution point i = sum_k i_k n^k (i_0 fastest); flux
 * point j = f N_fa + t on face f = 2k + s (s = 0: xi_k = -1, s = 1: xi_k = +1), t the index
 * of its tangential Gauss-Legendre positions, first tangential axis fastest. Triangles:
 * the point order of pcpf_triangle_operators (flux point j = e (p+1) + t, t along the walk
 * of edge e). */
typedef struct pcpf_dense_mesh {
    int32_t ndims;              /* d */
    int32_t order;              /* p */
    int32_t shape;              /* PCPF_SHAPE_* */
    int32_t nupts;              /* N_u: (p+1)^d for tensor elements, (p+1)(p+2)/2 for
                                   triangles */
    int32_t nfpts;              /* N_f: 2d (p+1)^(d-1) for tensor elements, 3(p+1) for
                                   triangles */
    int64_t nelem;              /* E */
    const double* M0;           /* [N_f][N_u] interpolation to the flux points (Step 1) */
    const double* D;            /* [d][N_u][N_u] reference derivatives (Steps 3, 6) */
    const double* LiftN;        /* [d][N_u][N_f] gradient correction, nhat_k-signed (Step 3) */
    const double* Lift;         /* [N_u][N_f] divergence correction (Step 6) */
    const double* Vinv;         /* [N_u][N_u] nodal -> orthonormal modal (sensor, §3.2) */
    const uint8_t* topmask;     /* [N_u] 1 on the modes dropped by the sensor's truncation */
    const double* W;            /* [N_u] quadrature weights of the solution points */
    const double* ref_fnorm;    /* [N_f][d] reference outward unit normal nhat_j */
    const double* jinv;         /* [E][d][d] J^-1, J = dx/dxi */
    const double* detj;         /* [E] det J */
    const double* fnorm;        /* [E][N_f][d] physical unit normal J^-T nhat / |J^-T nhat| */
    const double* fscale;       /* [E][N_f] det J |J^-T nhat| */
    const double* xorig;        /* [E][d] image of the reference corner (-1, ..., -1);
                                   of the vertex (0, 0) for triangles */
    const double* jac;          /* optional ([E][d][d] J itself; NULL: J = inv(jinv)) */
    const int32_t* nbr_slot;    /* [E N_f] partner flux point e' N_f + j', -1 = boundary
                                   (copy boundary condition, §3.3) */
    const uint8_t* owner;       /* [E N_f] 1 where this element computes the face's common
                                   flux (the side whose LDG beta is +1/2) */
    double period[3];           /* as pcpf_mesh.period */
} pcpf_dense_mesh;

typedef struct pcpf_ctx pcpf_ctx;

/* ABI version of the loaded library (PCPF_ABI_VERSION of its build). */
int pcpf_abi_version(void);

/* Message of the last failure of ctx, or of the calling thread's last failed call
 * when ctx is NULL (e.g. a failed pcpf_create). Never NULL; owned by the library. */
const char* pcpf_last_error(const pcpf_ctx* ctx);

/* --- host helpers (no GPU needed) -------------------------------------------------- */

/* 1D operators of the order-p Gauss-Legendre nodal element with DG (Radau) correction
 * functions (§3.1: Gauss-Legendre solution points, nodal basis from a Legendre
 * Vandermonde matrix). Each output is caller-owned host memory of the size given in
 * pcpf_mesh. EINVAL if order is outside 1..PCPF_MAX_ORDER or a pointer is NULL. */
pcpf_status pcpf_line_operators(int32_t order, double* nodes, double* weights,
                                double* deriv, double* lminus, double* lplus,
                                double* cminus, double* cplus, double* vinv);

/* Dense operators of the order-p triangle (§3.1 on triangles; the paper names the
 * Williams-Shunn solution points but prints no coordinates, so this library places them on
 * the interior lattice ((i + 1/3), (j + 1/3)) / (p + 1) of the reference triangle
 * {r, s >= 0, r + s <= 1}, j outer, i inner; p + 1 Gauss-Legendre flux points on each edge,
 * edges v0 -> v1, v1 -> v2, v2 -> v0 with v0 = (0, 0), v1 = (1, 0), v2 = (0, 1), each walked
 * in that direction; DG correction functions, Lift = M^-1 E). The arrays, host, float64,
 * caller-owned, have the shapes and meanings of pcpf_dense_mesh with N_u = (p+1)(p+2)/2,
 * N_f = 3 (p + 1), plus upt_ref [N_u][2] and fpt_ref [N_f][2], the reference coordinates of
 * the solution and flux points (a triangle element maps as x = xorig + J (r, s)).
 * EINVAL if order is outside 1..5 or a pointer is NULL. */
pcpf_status pcpf_triangle_operators(int32_t order, double* upt_ref, double* fpt_ref,
                                    double* M0, double* D, double* LiftN, double* Lift,
                                    double* Vinv, uint8_t* topmask, double* W,
                                    double* ref_fnorm);

/* Physical coordinates of every solution point, xs[(e*N_u + i)*d + k] (host, float64,
 * caller-owned, E*N_u*d values). EINVAL on a malformed mesh. */
pcpf_status pcpf_solution_coords(const pcpf_mesh* mesh, double* xs);

/* --- context ------------------------------------------------------------------------ */

/* Device workspace bytes a context needs for this mesh and form. */
pcpf_status pcpf_workspace_bytes(const pcpf_mesh* mesh, const pcpf_params* params,
                                 size_t* nbytes);

/* Validate mesh and parameters (sizes, det J > 0, reciprocal adjacency, matching face
 * points up to a translation), copy them to the device and create a context.
 * d_ws: caller-owned device memory of at least pcpf_workspace_bytes bytes, 256-byte
 * aligned, which must outlive the context. stream: a hipStream_t (NULL = default).
 * EINVAL, EUNSUPPORTED, EDEVICE. */
pcpf_status pcpf_create(const pcpf_mesh* mesh, const pcpf_params* params, void* d_ws,
                        size_t ws_bytes, void* stream, pcpf_ctx** out);

/* The dense description of pcpf_dense_mesh, validated and mapped onto the kernels' form.
 * The kernels apply the operators of a tensor-product element line by line (the sum-
 * factorised form of the same matrices), so the description is accepted when
 *   - its operators are those of the order-p Gauss-Legendre tensor element with DG
 *     correction functions in the point and face order stated above (each matrix entry
 *     within 1e-12 of the library's, relative to the operator's largest entry), and
 *   - every face is paired whole with the opposite face of one neighbour, flux point t
 *     with flux point t (the orientation rule of pcpf_mesh), owner = 1 exactly on the
 *     + faces of paired slots, and
 *   - the geometry is that of one affine map per element (det J, normals and face scales
 *     consistent with J^-1 within 1e-12).
 * Other point sets or orientations of tensor elements are valid descriptions that this
 * build does not run: EUNSUPPORTED. Inconsistent sizes, non-reciprocal pairs, several or no
 * owners on a pair, or geometry that disagrees with J: EINVAL.
 * Triangles (shape PCPF_SHAPE_TRIANGLE, d = 2, p = 1..5) run on dense per-element kernels:
 * the operators must be those of pcpf_triangle_operators (same tolerance), any pairing of
 * flux points is accepted when it is reciprocal, the paired points coincide (up to the
 * periods) and each pair has exactly one owner (boundary points are owned), and the map is
 * x = xorig + J (r, s). The common normal flux of a pair is computed once, by its owner,
 * as a physical flux; each side transforms it with its own fscale (the two sides of an edge
 * may sit on reference edges of different lengths). The adjoint and the BF16 form are not
 * built for triangles (EUNSUPPORTED). The host arrays are read during the call only.
 * pcpf_workspace_bytes_dense runs the same validation (no GPU needed); for tensor elements
 * pcpf_create_dense then behaves as pcpf_create on the equivalent pcpf_mesh. */
pcpf_status pcpf_workspace_bytes_dense(const pcpf_dense_mesh* mesh, const pcpf_params* params,
                                       size_t* nbytes);
pcpf_status pcpf_create_dense(const pcpf_dense_mesh* mesh, const pcpf_params* params,
                              void* d_ws, size_t ws_bytes, void* stream, pcpf_ctx** out);

/* Free the host-side context (the workspace stays with the caller). NULL is a no-op. */
void pcpf_destroy(pcpf_ctx* ctx);

/* Number of solution points per element and of elements. */
pcpf_status pcpf_sizes(const pcpf_ctx* ctx, int64_t* nelem, int32_t* nupts);

/* Set the state from device arrays [E][N_u] (state type). d_psi == NULL forces a reset +
 * preconditioning before the next step. t is the physical time, step the index of the
 * next step (resets happen before steps with step % reset_every == 0). */
pcpf_status pcpf_set_state(pcpf_ctx* ctx, const void* d_phi, const void* d_psi, double t,
                           int64_t step);

/* Copy the state out (either output may be NULL). Synchronous for t and step only. */
pcpf_status pcpf_get_state(pcpf_ctx* ctx, void* d_phi, void* d_psi, double* t,
                           int64_t* step);

/* Advance nsteps classic RK4 steps of size dt (§3.1 last paragraph), with the reset +
 * preconditioning of §2/§3.2 before each step whose index is a multiple of reset_every.
 * Synchronises the stream once at the end to read the non-finite flag: ENONFINITE if any
 * value became NaN/Inf or |phi| > 10 (the state is kept for inspection). Under
 * PCPF_STOP_RMS each pseudo-time iteration of a reset also reads its RMS back (one
 * synchronisation per iteration). */
pcpf_status pcpf_step(pcpf_ctx* ctx, double dt, int64_t nsteps);

/* Reset psi from the current phi (psi0 = phi - 1/2, or eps_w ln(phi/(1-phi)) with the
 * LOGIT mode, always in float64), compute the smeared sign tanh(psi0/max(|grad psi0|,
 * delta_g)) (PCPF_SGN_PSI0; PCPF_SGN_CURRENT keeps psi0 and takes |grad psi| at every
 * pseudo stage) and run iters pseudo-time RK4 iterations (iters < 0:
 * params.precond_iters), stopping early under PCPF_STOP_RMS. phi is not changed.
 * PCPF_STOP_RMS reads one double back per iteration (a stream synchronisation). */
pcpf_status pcpf_precondition(pcpf_ctx* ctx, int32_t iters);

/* The last preconditioning (pcpf_precondition or a reset inside pcpf_step): the number of
 * pseudo-time iterations it ran and, under PCPF_STOP_RMS, the RMS of (psi^k -
 * psi^(k-1)) / dtau after the last of them (NaN under PCPF_STOP_FIXED). Either output may
 * be NULL. ESTATE before the first preconditioning. */
pcpf_status pcpf_precond_info(const pcpf_ctx* ctx, int32_t* iters, double* rms);

/* One residual evaluation (the parity entry point). PCPF_MODE_PHYS: d/dt of (phi, psi)
 * at time t from d_phi, d_psi into d_rphi, d_rpsi: the FR residual of §3.1 (Steps 1-6,
 * du/dt = -div f / det J) of the localized system of §2 (Eq. altconservativephasefieldeq
 * for phi, the transport of psi). PCPF_MODE_PRECOND: d/dtau of psi (§3.2, Eq.
 * pseudotimesystem: the viscous flux with the sensor's nu_s plus the eikonal source) from
 * d_psi using the smeared sign of the last reset (d_phi, d_rphi ignored, may be NULL).
 * Inputs and outputs are [E][N_u] in the state type; outputs may not alias inputs.
 * Uses the context's scratch registers: the stored state is not changed. */
pcpf_status pcpf_residual(pcpf_ctx* ctx, const void* d_phi, const void* d_psi, double t,
                          int32_t mode, void* d_rphi, void* d_rpsi);

/* Smeared sign of the last reset, [E][N_u] in the state type (under PCPF_SGN_CURRENT:
 * psi0, from which each pseudo stage forms the sign). ESTATE before a reset. */
pcpf_status pcpf_get_sign(pcpf_ctx* ctx, void* d_sgn);

/* Persson-Peraire element viscosity nu_s (§3.2, Eqs. resolutionIndicator and nu_s) of the
 * field d_psi [E][N_u] into d_nu [E] (state type). */
pcpf_status pcpf_sensor(pcpf_ctx* ctx, const void* d_psi, void* d_nu);

/* FP64 reductions with the element quadrature |J| W (§4 error measures):
 * PCPF_REDUCE_MASS: integral of d_field (NULL: the stored phi);
 * PCPF_REDUCE_L1:   integral of |d_field - d_ref| (d_field NULL: the stored phi);
 * PCPF_REDUCE_RMS:  sqrt(sum over all E N_u points of (d_field - d_ref)^2 / (E N_u)),
 *                   unweighted (the norm of the pseudo-time stop rule, §3.2).
 * Deterministic two-pass reduction; synchronous (8 bytes device to host). EINVAL for an
 * unknown kind or a missing d_ref. */
pcpf_status pcpf_reduce(pcpf_ctx* ctx, int32_t what, const void* d_field,
                        const void* d_ref, double* out);

/* --- measurement -------------------------------------------------------------------- */

/* Kernel classes of the per-launch timing. */
enum { PCPF_KT_GRAD_FLUX = 0,     /* physical grad_flux launches (Steps 1-5)           */
       PCPF_KT_UPDATE = 1,        /* physical update launches (Step 6 + RK4 combine)   */
       PCPF_KT_PC_GRAD_FLUX = 2,  /* preconditioning grad_flux launches               */
       PCPF_KT_PC_UPDATE = 3,     /* preconditioning update launches                  */
       PCPF_KT_COUNT = 4 };

/* on != 0: pcpf_step and pcpf_precondition record a HIP event pair around every
 * grad_flux / update launch on the context's stream and accumulate the elapsed times
 * when they synchronise. Off by default (the event records add a small gap between
 * launches). */
pcpf_status pcpf_set_timing(pcpf_ctx* ctx, int32_t on);

/* Accumulated kernel time in milliseconds and launch count per class, host arrays of
 * PCPF_KT_COUNT entries (either may be NULL); reset != 0 clears the accumulators. */
pcpf_status pcpf_kernel_times(pcpf_ctx* ctx, double* ms, int64_t* launches, int32_t reset);

/* --- adjoint (reverse mode) ----------------------------------------------------------
 *
 * Gradients of a loss L(phi(T), psi(T)) of the discrete solution after nsteps RK4 steps
 * with respect to the initial state and to the velocity amplitude A (v = A v0(x) g(t)):
 * the exact vector-Jacobian products of the discrete scheme above (the FR operators of
 * §3.1 applied transposed, the fluxes of §2 and the preconditioner of §3.2 differentiated
 * by hand), including every reset + preconditioning inside the run. The forward run is
 * checkpointed every `every` steps and each segment is recomputed once in the reverse
 * sweep (every stage input of the segment is held in the scratch buffer).
 */

/* Set the velocity amplitude A of subsequent calls (the adjoint's parameter). */
pcpf_status pcpf_set_velocity_amplitude(pcpf_ctx* ctx, double amp);

/* Bytes of the checkpoint buffer of a run of nsteps steps checkpointed every `every`
 * steps: ceil(nsteps / every) copies of (phi, psi). EINVAL unless nsteps >= 1 and
 * every >= 1. */
pcpf_status pcpf_ckpt_bytes(const pcpf_ctx* ctx, int64_t nsteps, int64_t every,
                            size_t* nbytes);

/* Advance the stored state by nsteps steps exactly as pcpf_step does, keeping (phi, psi)
 * before every step whose index (counted from this call) is a multiple of `every` in
 * d_ckpt (caller-owned device memory of pcpf_ckpt_bytes bytes). Records the run (start
 * time and step, dt, nsteps, every, A, whether psi was set) for pcpf_adjoint. When resets
 * are scheduled, every <= reset_every is required (at most one reset per segment), and a
 * run that starts without psi must start on the reset schedule. Synchronous. ESTATE
 * without a state, EINVAL, ENONFINITE (the run is then not recorded), EUNSUPPORTED for
 * the PCPF_BF16 form and for PCPF_NORMAL_PHI (the adjoint kernels differentiate the
 * FP64 and FP32 forms of the method with the psi normal). */
pcpf_status pcpf_forward_ckpt(pcpf_ctx* ctx, double dt, int64_t nsteps, int64_t every,
                              void* d_ckpt, size_t ckpt_bytes);

/* Device scratch bytes pcpf_adjoint needs for checkpoints every `every` steps
 * (4 stage inputs of every step of one segment, the stage inputs of one preconditioning,
 * and the adjoint registers). */
pcpf_status pcpf_adjoint_bytes(const pcpf_ctx* ctx, int64_t every, size_t* nbytes);

/* Reverse sweep of the last pcpf_forward_ckpt run (d_ckpt unchanged since), with the
 * amplitude A recorded by that run.
 * d_gphi, d_gpsi: dL/dphi(T), dL/dpsi(T) ([E][N_u], state type; d_gpsi may be NULL = 0).
 * Outputs: d_gphi0 = dL/dphi(0), d_gpsi0 = dL/dpsi(0) (may be NULL; zero when the run
 * started with a reset, which discards psi(0)), *g_amp = dL/dA (may be NULL, float64,
 * deterministic). d_scratch: caller-owned, 256-byte aligned, >= pcpf_adjoint_bytes.
 * The stored state is used as a recompute register: after the call no state is set
 * (ESTATE until pcpf_set_state). Synchronous. ESTATE without a recorded run, EINVAL. */
pcpf_status pcpf_adjoint(pcpf_ctx* ctx, const void* d_ckpt, void* d_scratch,
                         size_t scratch_bytes, const void* d_gphi, const void* d_gpsi,
                         void* d_gphi0, void* d_gpsi0, double* g_amp);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): pcpf_adjoint with its scratch taken
 * from a static array the library holds on each GPU it runs on (PCPF_ADJOINT_STATIC_BYTES,
 * kept until the process ends) instead of caller memory. Same arguments and results as
 * pcpf_adjoint otherwise, and the same kernels; it calls no allocating routine (per-launch
 * timing is suspended during the call, since it creates events). The context's GPU must be
 * current. EINVAL when the run needs more scratch than the static array
 * (pcpf_adjoint_bytes > PCPF_ADJOINT_STATIC_BYTES; checkpoint more often or use
 * pcpf_adjoint). All calls on one GPU share its array: calls that overlap in time on one
 * GPU (two threads, or two streams whose work overlaps) race and give wrong gradients;
 * serialise them. Every region the sweep accumulates into is cleared at the start of each
 * call. */
#define PCPF_ADJOINT_STATIC_BYTES (64u << 20)
pcpf_status pcpf_adjoint_static(pcpf_ctx* ctx, const void* d_ckpt, const void* d_gphi,
                                const void* d_gpsi, void* d_gphi0, void* d_gpsi0,
                                double* g_amp);

#ifdef __cplusplus
}
#endif
#endif /* PCPF_H */
