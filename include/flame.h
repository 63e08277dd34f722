/*
 * flame.h - C ABI of the MI355X library for the coupled Hall-MHD lattice-Boltzmann step
 * (Foldes et al., "Efficient kinetic Lattice Boltzmann simulation of three-dimensional
 * Hall-MHD turbulence", Sec. 3 and App. A-B).
 *
 * One step updates, at every node of a periodic nx x ny x nz grid (lattice units,
 * dx = dt = 1):
 *   - D3Q27 fluid populations f_i with the central-moment collision of Sec. 3.1.2 towards
 *     the sixth-order Hermite equilibrium upgraded by the Maxwell stress (App. A);
 *   - D3Q7 vector magnetic populations g_i (7 x 3) with the BGK collision of Sec. 3.2
 *     towards the Hall equilibrium (eq. gHall_eq), J taken either from the magnetic
 *     moments (eq. soe_current_density) or from the central-difference curl of B;
 *   - streaming of both sets along their lattice velocities.
 * Relaxation rates follow the paper: 1/omega = 3 nu + 1/2, 1/omega_B = 4 eta + 1/2.
 * Variants selected in flame_params: the BGK fluid collision (S = omega I), the
 * electron-MHD magnetic equilibrium (Sec. 6) and the other velocity sets of the lattice figure of
 * Sec. 3.1 (D3Q19 fluid, D3Q15 / D3Q27 magnetic). Diagnostics: FP64 reductions, shell energy and
 * dissipation spectra, and the energy transfer terms of the scale-by-scale budget (Sec. 4.4).
 *
 * Conventions shared by every entry point
 *   - Node index: cell = (z * ny + y) * nx + x.
 *   - Canonical population order: fluid i = 0..26 in the App. A listing of c_i; magnetic
 *     directions rest, -x, -y, -z, +x, +y, +z, each with components x, y, z.
 *     A canonical population array is double [27][nz][ny][nx] followed by
 *     double [7][3][nz][ny][nx] (48 * ncell doubles), holding the post-streaming,
 *     pre-collision values of the current time (full values, not deviations). On the lattice
 *     variants (FLAME_FLUID_*, FLAME_MAGNETIC_* below) it is [q][...] then [m][3][...].
 *   - Vector fields are double [3][nz][ny][nx]; gradients double [3][3][nz][ny][nx] with
 *     grad[a][b] = d field_b / d x_a.
 *   - "device" pointers are HIP device memory of the device current when flame_init was
 *     called; "host" pointers are ordinary host memory. The caller owns every buffer it
 *     passes; the library never frees caller memory.
 *   - All device work is enqueued on the stream given to flame_init, in order. Entry
 *     points that return host data synchronise that stream first; asynchronous kernel
 *     failures surface there as FLAME_E_HIP.
 *   - Status codes: 0 OK, negative = error (nothing was enqueued unless stated),
 *     positive = warning flags (the call completed).
 *   - A context is not thread-safe; calls on one context must not overlap.
 *   - Launch-shape tuning, read from the environment by flame_init (results do not depend on
 *     it, bitwise): FLAME_ZCHUNK_PLANES = planes per workgroup of the curl-stencil kernel
 *     (default 32), FLAME_ROW_THREADS = threads per row block of the node-local kernels, a
 *     multiple of 64 up to 256, larger values taken as 256 (default: the row rounded up to
 *     whole wavefronts, at most 256),
 *     FLAME_GLOBAL_ADDRESSING = 1 makes the node-local step of the paper's velocity sets address
 *     its arrays with 64-bit global addresses (default: buffer resources for FP16 and FP64
 *     storage wherever every array ends at least 16 bytes below 4 GiB).
 */
#ifndef FLAME_H
#define FLAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t flame_status;
#define FLAME_OK 0
#define FLAME_E_INVAL (-1)       /* invalid argument; message in flame_last_error */
#define FLAME_E_NOMEM (-2)       /* library scratch allocation failed */
#define FLAME_E_HIP (-3)         /* a HIP / hipFFT call failed (message names it) */
#define FLAME_E_NONFINITE (-4)   /* a population is NaN or infinite (flame_reduce) */
#define FLAME_E_UNSUPPORTED (-5) /* option combination not built */
#define FLAME_E_UNSTABLE (-6)    /* finite, but max|u| >= c_s = 1/sqrt(3): the run has left the
                                    weakly compressible regime the scheme is built for (flame_reduce) */
#define FLAME_W_CFL 1            /* advisory whistler bound pi * d_i * max|B| > 1 exceeded */

/* Storage precision of the populations. Values are stored as deviations from the rest
 * state f^mhd(0)(1, 0, b0), g = W_i b0; F16 additionally scales each deviation by an exact
 * power of two per velocity class. Collision arithmetic is FP64 for F64, FP32 otherwise. */
#define FLAME_F64 0
#define FLAME_F32 1
#define FLAME_F16 2

/* How J enters the Hall equilibrium. */
#define FLAME_J_MOMENT 0   /* 3x3 solve from the magnetic first moment (Sec. 3.2) */
#define FLAME_J_STENCIL 1  /* central-difference curl of B over the six face neighbours */

/* Population layout in the caller's storage buffer.
 * AB: two lattices for each set, pull streaming (a step reads population i of node x at
 *     x - c_i in one copy and writes it at x in the other).
 * AA: one lattice updated in place (even/odd step addressing); with FLAME_J_STENCIL the
 *     magnetic set keeps two lattices so that neighbour fields are read-only in a step. */
#define FLAME_LAYOUT_AB 0
#define FLAME_LAYOUT_AA 1

/* Fluid collision. CENTRAL is the paper's central-moment collision (Sec. 3.1.2,
 * S = diag[1,1,1,1,omega x5,1 x18]); BGK is the standard single-rate operator of Sec. 3.1.1,
 * the same step with S = omega I (every central moment relaxed at omega, the body force still
 * ending the first central moments at +F/2). */
#define FLAME_COLLISION_CENTRAL 0
#define FLAME_COLLISION_BGK 1

/* Magnetic equilibrium. HALL is eq. gHall_eq with V = U - alpha_H J; EMHD is the electron-MHD
 * variant of Sec. 6, with the bulk velocity neglected against the Hall current (V = -alpha_H J)
 * in the equilibrium, in the J system of the moment route and in the initial state. */
#define FLAME_MAGNETIC_HALL 0
#define FLAME_MAGNETIC_EMHD 1

/* Velocity sets (the lattice figure of Sec. 3.1; Sec. 4.3 reports runs with the larger magnetic
 * sets). The paper's are D3Q27 for the fluid and D3Q7 for the magnetic field (0, the defaults).
 * D3Q19 fluid: the App. A listing without its eight corners (directions 0..9 and 14..22 of it),
 *   weights 1/3, 1/18, 1/36; it runs the BGK collision (FLAME_COLLISION_BGK) towards the
 *   second-order Hermite equilibrium with the Maxwell-stress term, a body force entering as the
 *   second-order form w_i [(c_i - U)/c_s^2 + (c_i . U) c_i / c_s^4] . F of the D3Q27 force term.
 * D3Q15 / D3Q27 magnetic: W = 5/12, 1/12 (faces), 1/96 (corners), resp. 17/36, 1/18, 1/72
 *   (edges), 1/288 (corners): the fluid weights of the same velocities with the moving ones scaled
 *   by C^2 / c_s^2 = 3/4, which keeps sum W xi xi = C^2 I with C^2 = 1/4 (node coincidence,
 *   Sec. 3.2) and fourth-order isotropy. D3Q15 order: rest, -x, -y, -z, (-1,-1,-1), (-1,-1,1),
 *   (-1,1,-1), (-1,1,1), then the opposites of those seven in the same order; magnetic D3Q27
 *   takes the App. A order.
 * The lattice variants run the moment route of J (FLAME_J_MOMENT) in either layout, forward
 * only (the reverse-mode and trace entry points return FLAME_E_UNSUPPORTED). A canonical
 * population array then holds q fluid and m x 3 magnetic arrays (q = 27 or 19, m = 7, 15 or 27)
 * in the orders above. */
#define FLAME_FLUID_D3Q27 0
#define FLAME_FLUID_D3Q19 1
#define FLAME_MAGNETIC_D3Q7 0
#define FLAME_MAGNETIC_D3Q15 1
#define FLAME_MAGNETIC_D3Q27 2

/* Reduction slots of flame_reduce (FP64):
 *  0 E_kin = 1/2 <|u|^2>        1 E_mag = 1/2 <|B - b0|^2>     2 H_c = <u . (B - b0)>
 *  3 <|J|^2>                    4 max |div B|                  5 rms div B
 *  6 max |u|                    7 rms (rho - 1)                8 nodes with a non-finite value
 *  9 sum rho                   10-12 sum rho u                13-15 sum B
 * div B is the moment estimate -(omega_B / C^2) Tr Lambda of eq. LB_B_div; <.> is the node
 * average. u and B include the forcing half-shifts F/(2 rho) and S/2. */
#define FLAME_NRED 16

typedef struct {
  int32_t nx, ny, nz;   /* grid; each >= 1 (>= 3 with FLAME_J_STENCIL), nz <= 65535; one population
                           array (nx*ny*nz values, padded to 256 bytes) and, when forcing is
                           given, one forcing array must each span at most 4 GiB */
  double nu;            /* lattice kinematic viscosity, > 0 */
  double eta;           /* lattice resistivity, > 0 */
  double d_i;           /* Hall coefficient alpha_H in cells (ion inertial length, rho0 = 1), >= 0 */
  double b0[3];         /* uniform background field */
  int32_t storage;      /* FLAME_F64 / FLAME_F32 / FLAME_F16 */
  int32_t jmode;        /* FLAME_J_MOMENT / FLAME_J_STENCIL */
  int32_t layout;       /* FLAME_LAYOUT_AB / FLAME_LAYOUT_AA */
  int32_t init_noneq;   /* 1: add the first-order non-equilibrium parts at initialisation */
  /* Optional static body force F on the fluid and solenoidal source S on the field
   * (device, [3][nz][ny][nx], double for FLAME_F64 and float otherwise, nullable; must
   * stay valid while the context lives). Each step adds F to the momentum and S to B. */
  const void* force_u;
  const void* force_b;
  int32_t collision;    /* FLAME_COLLISION_CENTRAL (0, the paper's) / FLAME_COLLISION_BGK */
  int32_t magnetic;     /* FLAME_MAGNETIC_HALL (0, the paper's) / FLAME_MAGNETIC_EMHD; the reverse-mode
                           and trace entry points accept only the defaults (FLAME_E_UNSUPPORTED) */
  int32_t fluid_lattice;     /* FLAME_FLUID_D3Q27 (0, the paper's) / FLAME_FLUID_D3Q19 */
  int32_t magnetic_lattice;  /* FLAME_MAGNETIC_D3Q7 (0, the paper's) / _D3Q15 / _D3Q27 */
} flame_params;

typedef struct flame_ctx flame_ctx;

/* Bytes of population storage the caller must provide for these parameters (0 if the
 * parameters are invalid). AB: 96 values per node; AA: 48 (69 with FLAME_J_STENCIL);
 * values are 8, 4 or 2 bytes. On lattice variants: q + 3 m values per node (AA), twice that (AB).
 * FLAME_E_UNSUPPORTED combinations (a lattice variant with the stencil route, D3Q19 with the
 * central-moment collision) give 0 as well. */
size_t flame_storage_bytes(const flame_params* p);

/* Rest state the stored deviations are measured from (host, no device use):
 * f_rest[q] = f^mhd(0)(1, 0, b0) (App. A equilibrium with the Maxwell stress of b0) and
 * g_rest[3 m] = W_i b0 (index i * 3 + component); q = 27, m = 7 on the paper's lattices. Either
 * pointer may be NULL. */
flame_status flame_rest_populations(const flame_params* p, double* f_rest, double* g_rest);

/* Create a context over caller-owned population storage and fill it with the initial state
 * (paper: rho = 1 everywhere, Sec. 4.1): f = f^mhd(0)(1, u, B), g = g^Hall(0)(u, B, curl B),
 * plus, if init_noneq and the gradients are given, the first-order non-equilibrium parts
 * (deviatoric stress -(c_s^2/omega)(grad u + grad u^T - 2/3 div u I) and magnetic
 * -(1/omega_B) W_i xi_ia d_a B_b). With forcing, -F/2 and -S/2 shifts make the node moments
 * return exactly u and B = b0 + b.
 *   u, b: device double [3][nz][ny][nx] (velocity; field fluctuation, B = b0 + b).
 *   grad_u, grad_b: device double [3][3][nz][ny][nx] or NULL. A NULL gradient is replaced,
 *     when init_noneq is set, by the central difference of u (or b) on the grid,
 *     (v(x + e_a) - v(x - e_a)) / 2; without init_noneq a NULL grad_b gives J = 0 in the initial
 *     Hall equilibrium and no non-equilibrium part is added.
 *   storage: device, at least flame_storage_bytes(p) bytes, 256-byte aligned.
 *   hip_stream: hipStream_t (NULL = default stream).
 * Returns FLAME_OK or FLAME_W_CFL with *out set; on error *out is NULL. */
flame_status flame_init(const flame_params* p, const double* u, const double* b,
                        const double* grad_u, const double* grad_b, void* storage,
                        size_t storage_bytes, void* hip_stream, flame_ctx** out);

/* Advance nsteps >= 0 time steps, asynchronously: per step one fused kernel launch that
 * collides (Sec. 3.1.2 fluid, Sec. 3.2 magnetic) and streams (eq. stream) every node. */
flame_status flame_step(flame_ctx* c, int64_t nsteps);

/* Node fields of the current state into nullable device double buffers:
 * rho [nz][ny][nx]; u, b (full B), j [3][nz][ny][nx]; divb [nz][ny][nx]. J is the one the
 * next step would use (moment or stencil route). Asynchronous. */
flame_status flame_moments(flame_ctx* c, double* rho, double* u, double* b, double* j,
                           double* divb);

/* FP64 global reductions (slots above) into host out[FLAME_NRED]. Synchronises. Returns
 * FLAME_E_NONFINITE (after filling out) if any population is non-finite, else
 * FLAME_E_UNSTABLE (after filling out) if max|u| (slot 6) reaches the lattice sound speed
 * c_s = 1/sqrt(3): the equilibria of Sec. 3.1 are expansions in the Mach number, and a flow at
 * Mach one is a blow-up, not a solution. Fixed-order tree sums and a fixed-order merge of the
 * block partials: bitwise reproducible for a given grid and state. */
flame_status flame_reduce(flame_ctx* c, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the reductions of flame_reduce, computed by the same
 * kernels in the same fixed order (bitwise the same values), into a caller-owned device buffer
 * out[FLAME_NRED] (double), asynchronously on the context's stream. Allocates nothing and does
 * not synchronise: the block partials go to a static device array of 2048 x FLAME_NRED doubles
 * (256 KiB per GPU, held until the process ends), which covers every grid (the reduction visits
 * the nodes with at most 2048 blocks). Calls on one GPU share that array and leave their partials
 * in it: calls that may overlap on one GPU (several streams or contexts) race and must be
 * ordered by the caller. There is no status for a blown-up state: slot 8 counts non-finite nodes
 * and slot 6 holds max|u| (FLAME_E_UNSTABLE at c_s = 1/sqrt(3) in flame_reduce).
 * FLAME_E_INVAL for a NULL out. */
flame_status flame_reduce_noalloc(flame_ctx* c, double* out);

/* Shell energy spectrum of u (field = 0) or B (field = 1) into host e_k[nshells]:
 * E(s) = 1/2 sum_{round(|k|) = s} |v_hat(k)|^2, v_hat = DFT(v) / ncell, k the signed integer
 * wavevector (paper Sec. 4.4 spectra). FP64 FFT (hipFFT) and binning in a fixed order (no
 * atomics), so the spectrum of a given state is bitwise reproducible. Synchronises. The first
 * call allocates a workspace of one node field and one half spectrum (kept until flame_destroy);
 * FLAME_E_NOMEM if that fails, and a later call tries again. */
flame_status flame_spectrum(flame_ctx* c, int32_t field, int32_t nshells, double* e_k);

/* Shell dissipation spectrum of u (field = 0) or B (field = 1) into host d_k[nshells]:
 * D(s) = sum_{round(|k|) = s} |q(k)|^2 |v_hat(k)|^2, q_a = 2 pi k_a / n_a in inverse cells, the
 * summand of the dissipation D(k) of the paper's scale-by-scale energy budget (Sec. 4.4, eq.
 * mhd_en_trans) without the factor nu or eta. sum_s D(s) = <|grad v|^2> (Parseval), which is
 * <|curl v|^2> for a solenoidal field, so nu sum D_u + eta sum D_B is the dissipation rate of
 * the energy 1/2 <|u|^2 + |B|^2>. Same transform, shells, errors (FLAME_E_INVAL for a field
 * other than 0 or 1, nshells outside 1..4096 or a NULL d_k) and synchronisation as
 * flame_spectrum. */
flame_status flame_dissipation_spectrum(flame_ctx* c, int32_t field, int32_t nshells, double* d_k);

/* Energy transfer terms of the scale-by-scale energy budget (paper Sec. 4.4, eq. mhd_en_trans)
 * per shell s = round(|k|), into host arrays of nshells each:
 *   t_adv[s] =  sum Re[u_hat* . F(U . grad U)],   t_lor[s] = -sum Re[u_hat* . F(J x B)],
 *   t_ind[s] = -sum Re[B_hat* . F(curl(U x B))],
 * and, when t_hall is not NULL, the Hall term of the induction equation, which the paper's flux
 * leaves out: t_hall[s] = +d_i sum Re[B_hat* . F(curl(J x B))] (it sums to zero over all shells
 * for J = curl B: the Hall term moves energy between scales without changing its total),
 * with F = DFT / ncell, U and B the node fields and J the current of the context's route (from
 * the magnetic moments, or the curl stencil). The flux across k is
 * S_MHD(k) = sum_{s < k} (t_adv + t_lor + t_ind); for incompressible MHD without Hall and pressure
 * terms, d/dt sum_{s < k} E(s) = -S_MHD(k) - D(k) with D from flame_dissipation_spectrum (with the
 * Hall term, -sum_{s < k} t_hall is added to the right-hand side).
 * Derivatives are spectral, q_a = 2 pi k_a / n_a, and 0 on the Nyquist index of an even axis;
 * products are formed node by node. FP64 throughout (hipFFT), shell sums in a fixed order
 * (bitwise reproducible for a given state). Allocates 11 node fields and 7
 * half spectra of device memory for the call (19 GB at 512^3) and frees them before returning;
 * FLAME_E_NOMEM if that fails. FLAME_E_INVAL for nshells outside 1..4096 or a NULL t_adv, t_lor
 * or t_ind. Synchronises. */
flame_status flame_energy_transfer(flame_ctx* c, int32_t nshells, double* t_adv, double* t_lor, double* t_ind,
                                   double* t_hall);

/* Copy the state in canonical order to / from device double dst/src [48 * ncell]
 * ([(q + 3 m) * ncell] on lattice variants).
 * deviations = 0: full population values; deviations = 1: departures from the rest state of
 * flame_rest_populations, which are the stored values exactly (decoded), so a get / set pair
 * with deviations = 1 restores a bitwise-identical state (checkpoint / resume).
 * flame_set_populations may be called at any time; it leaves the context at an even step and
 * resets the step count to 0. Both are asynchronous. */
flame_status flame_get_populations(flame_ctx* c, double* dst, int32_t deviations);
flame_status flame_set_populations(flame_ctx* c, const double* src, int32_t deviations);

/* Canonical populations of n given nodes: cells (device int64 [n], linear node indices)
 * -> out (device double [n][48]: 27 fluid then 7 x 3 magnetic ([n][q + 3 m] on lattice
 * variants); full values or deviations as
 * above; NaN rows for indices outside the grid). Asynchronous. */
flame_status flame_gather(flame_ctx* c, const int64_t* cells, int64_t n, double* out,
                          int32_t deviations);

/* ---- Reverse mode (adjoint of the step; not part of the paper's method) ----------------------
 * Arrays below are in the arithmetic type A (double for FLAME_F64, float otherwise), canonical
 * order, node stride n = nx*ny*nz: "state" [48 + 3][n] = pre-collision deviations (27 fluid,
 * 7 x 3 magnetic) followed by the J each node used; "lam" [48][n] = d loss / d(canonical
 * deviations) at one time. All are device pointers, caller-owned, asynchronous. The kernels
 * address each [n] array with 32-bit byte offsets: flame_step_save, flame_adjoint_step and
 * flame_adjoint_trace_step return FLAME_E_INVAL when n values of A exceed 4 GiB. */

/* One step, like flame_step(c, 1), that also writes the state it advanced from into state. */
flame_status flame_step_save(flame_ctx* c, void* state);

/* lam = (d step / d x)^T lam_next at the state saved by flame_step_save: the gather that
 * transposes streaming, then the reverse pass of every node's collision (moments, J on the
 * moment route, central-moment fluid and Hall magnetic collisions, forcing). On the stencil
 * route lam_j ([3][n] scratch) receives d loss / dJ and its transpose-curl is added to the
 * magnetic adjoints. lam must not alias lam_next. */
flame_status flame_adjoint_step(flame_ctx* c, const void* state, const void* lam_next, void* lam,
                                void* lam_j);

/* Trace lattices (moment route, AA layout): one time level laid out as a two-lattice pull
 * source, 48 arrays [q][n] of the storage type (27 fluid, then 7 x 3 magnetic), node stride
 * n = nx*ny*nz, with the stored encoding of the deviations; slot q at node y holds the
 * post-collision population q of node y, so population q of node x at the next step is slot q
 * at x - c_q. flame_trace_bytes(c) bytes each (0 if c is NULL or runs a model or velocity-set
 * variant, which have no trace lattice). flame_trace_export writes the
 * current state (exact: stored values are moved, not recoded); flame_trace_step advances a
 * lattice src by one step into dst (dst must not alias src) without touching the context, and
 * reproduces the context's own steps bitwise. Other routes and layouts (the stencil route, the AB
 * layout) get FLAME_E_UNSUPPORTED from all three calls that take a lattice, and nothing is
 * launched. */
size_t flame_trace_bytes(const flame_ctx* c);
flame_status flame_trace_export(flame_ctx* c, void* lat);
flame_status flame_trace_step(flame_ctx* c, const void* src, void* dst);

/* Moment route: lam = (d step / d x)^T lam_next for the step whose pre-collision state is the
 * trace lattice src pulled (the step flame_trace_step takes from src), with J recomputed from
 * that state; the same reverse pass as flame_adjoint_step without a saved state. lam, lam_next
 * as for flame_adjoint_step; lam must not alias lam_next. The stencil route and the AB layout get
 * FLAME_E_UNSUPPORTED. */
flame_status flame_adjoint_trace_step(flame_ctx* c, const void* src, const void* lam_next, void* lam);

/* lam = adjoint of the current state for a loss of its node fields: dl_du, dl_db (device
 * double [3][n], nullable = zero) are d loss / du and d loss / dB with u, B as flame_moments
 * returns them. */
flame_status flame_adjoint_fields(flame_ctx* c, const double* dl_du, const double* dl_db, void* lam);

/* Adjoint of the initial state of flame_init: from lam0 (d loss / d initial deviations) and the
 * same u, b, grad_u, grad_b that flame_init received, write g_u, g_b (device double [3][n]) and,
 * when non-NULL, g_grad_u, g_grad_b ([3][3][n]). With init_noneq both gradients must be given
 * (FLAME_E_UNSUPPORTED otherwise: the transpose of the internal central differences is not
 * built). */
flame_status flame_adjoint_init(flame_ctx* c, const void* lam0, const double* u, const double* b,
                                const double* grad_u, const double* grad_b, double* g_u, double* g_b,
                                double* g_grad_u, double* g_grad_b);

/* Number of steps taken since flame_init / flame_set_populations. */
int64_t flame_step_count(const flame_ctx* c);

/* Advisory whistler CFL number pi * d_i * max|B| of the initial state. */
double flame_cfl_number(const flame_ctx* c);

/* Message of the last error on this context ("" if none); c may be NULL for errors from
 * flame_init. The pointer stays valid until the next call on the context. */
const char* flame_last_error(const flame_ctx* c);

/* Release the context and the library's scratch buffers (never the caller's storage).
 * Synchronises the stream first. */
void flame_destroy(flame_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* FLAME_H */
