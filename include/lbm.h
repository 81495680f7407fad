/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library.
 *
 * The library advances the fused collide-and-stream update of the two
 * collision models compared by Geller, Uphoff & Krafczyk, "Turbulent jet
 * computations based on MRT and Cascaded Lattice Boltzmann models"
 * (arXiv:1206.0389):
 *   - D3Q19 MRT with a Smagorinsky eddy viscosity (Section 2, Eq. (12),
 *     Table 1, Eqs. (16)-(21));
 *   - D3Q27 factorized cascaded LB, FCLB (Section 2, Eqs. (14)-(15),
 *     Table 2), with no explicit turbulence model.
 * Populations live in device memory as deviations f_i - w_i from the rest
 * equilibrium, stored in FP64, FP32 or FP16; arithmetic runs in FP64 for
 * FP64 storage and in FP32 otherwise; global sums always run in FP64.
 *
 * Conventions shared by every call
 *   - Population order at the ABI is the order of the velocity tables of
 *     Section 2 (D3Q27 indices 0..18 coincide with D3Q19).
 *   - Field layout: x fastest, then y, then z. Scalar fields have nx*ny*nz
 *     entries; vector fields are [3][nz][ny][nx]; population fields are
 *     [Q][nz][ny][nx].
 *   - All pointers marked "device" must be device memory of the current HIP
 *     device (for example a torch tensor's data pointer). The caller owns
 *     every buffer; the library never allocates device memory, it only
 *     uses the block handed over by lbm_bind_memory.
 *   - Calls are asynchronous on the stream given in lbm_config (or set by
 *     lbm_set_stream), except where a call is documented as blocking.
 *   - Every call returns LBM_OK (0) or a negative status. Arguments are
 *     validated before anything is launched; a failing call changes
 *     nothing. lbm_strerror() gives a message; for LBM_EHIP it returns the
 *     HIP error text of the last failure on the calling thread.
 *   - A lattice handle must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)      /* bad argument or configuration            */
#define LBM_ENOMEM (-2)      /* bound block smaller than required         */
#define LBM_EUNBOUND (-3)    /* no device memory bound yet                */
#define LBM_EHIP (-4)        /* a HIP call or launch failed               */
#define LBM_ENONFINITE (-5)  /* a global sum is NaN or infinite           */
#define LBM_ESTATE (-6)      /* call not valid in the lattice's state     */
#define LBM_EMASS (-7)       /* mass drift beyond the lbm_set_check bound */

/* ---- enumerations ----------------------------------------------------- */
#define LBM_D3Q19_MRT_LES 1  /* Eq. (12) + Eqs. (16)-(21), incompressible */
#define LBM_D3Q27_FCLB 2     /* Table 2 central moments, compressible     */
#define LBM_D3Q27_CLB 3      /* cascaded, Gaussian higher-order equilibria */

#define LBM_F64 1            /* population storage types                  */
#define LBM_F32 2
#define LBM_F16 3

#define LBM_DTYPE_F64 1      /* element type of caller field buffers      */
#define LBM_DTYPE_F32 2

#define LBM_BASIS_TABLE1 0   /* MRT moments grouped as in Table 1         */
#define LBM_BASIS_DHUMIERES 1 /* d'Humieres et al. (2002) orthogonal basis */

#define LBM_PERIODIC 0       /* face types                                */
#define LBM_WALL 1           /* halfway bounce-back, optional velocity    */
#define LBM_INLET 2          /* halfway bounce-back with inlet velocity   */
#define LBM_OUTFLOW 3        /* zero-gradient: ghost copy of last plane   */
#define LBM_FREESLIP 4       /* halfway specular reflection (free slip)   */
#define LBM_PRESSURE 5       /* fixed pressure: anti-bounce-back          */

#define LBM_RHO_FULL 0       /* lbm_get_macroscopic: write rho            */
#define LBM_RHO_DEVIATION 1  /* ... write rho - 1                         */

typedef struct lbm_lattice lbm_lattice;

/*
 * Lattice configuration (copied at create; no pointer is kept).
 *   model      LBM_D3Q19_MRT_LES, LBM_D3Q27_FCLB or LBM_D3Q27_CLB (the
 *              cascaded scheme before the factorization, Section 2: the same
 *              central moments and rates as the FCLB, with the fourth- and
 *              sixth-order central moments relaxed to those of the Gaussian,
 *              rho/9, 0 and rho/27; no adjoint).
 *   storage    LBM_F64, LBM_F32 or LBM_F16 (population deviations).
 *   nx,ny,nz   lattice nodes, each >= 1; nx*ny*nz < 2^31.
 *   nu         lattice kinematic viscosity, > 0; the molecular relaxation
 *              time is tau0 = 3 nu + 1/2 (Eq. (13), c = 1), so omega =
 *              1/tau0 must be < 2.
 *   cs_smag    Smagorinsky constant C_S >= 0 (MRT only; 0 switches the
 *              eddy viscosity off). Eq. (20) gives tau_total.
 *   mrt_basis  LBM_BASIS_TABLE1 (the paper's choice) or LBM_BASIS_DHUMIERES.
 *   rates      non-shear relaxation rates, used when use_default_rates = 0:
 *              TABLE1: s2 (trace), s3, s4, s7 (all 4th-order rows);
 *              DHUMIERES: s_e, s_eps, s_q, s_pi, s_m.
 *              Defaults: TABLE1 all 1 (Section 2: s_i = 1 for i != 1);
 *              DHUMIERES 1.19, 1.4, 1.2, 1.4, 1.98.
 *              The FCLB model ignores them (all non-shear rates are 1).
 *   stream     hipStream_t for every asynchronous call (0 = null stream).
 */
typedef struct lbm_config {
  int32_t model;
  int32_t storage;
  int32_t nx, ny, nz;
  int32_t mrt_basis;
  double nu;
  double cs_smag;
  double rates[8];
  int32_t use_default_rates;
  int32_t reserved0;
  void* stream;
} lbm_config;

/*
 * Boundary description, one entry per face in the order
 * x-, x+, y-, y+, z-, z+ (the "-" face holds coordinate 0).
 *   face_type  LBM_PERIODIC | LBM_WALL | LBM_INLET | LBM_OUTFLOW |
 *              LBM_FREESLIP | LBM_PRESSURE (the last two on uniform
 *              lattices only). Opposite
 *              faces must both be periodic or both non-periodic.
 *              At most one LBM_INLET face and one LBM_OUTFLOW face; the
 *              outflow face must be a z face (z- or z+).
 *   face_u     wall velocity of LBM_WALL faces (lattice units).
 *   inlet_u    device, velocity on the inlet face, [3][nb][na] of
 *              inlet_dtype, where (a, b) are the face's two tangential
 *              coordinates in increasing axis order (z face: a = x, b = y).
 *   inlet_mask device uint8 [nb][na] or NULL; where 1, each component gets
 *              a seeded uniform perturbation inlet_amp * (2U - 1) drawn
 *              per time step from SplitMix64 of the seed xor the packed
 *              (t, component, b, a).
 *   seed       perturbation seed.
 * The streaming rule at a face (population i arriving from outside at
 * node x, post-collision values f*):
 *   WALL, INLET  f_i(x) = f*_opp(i)(x) + 6 w_i (e_i . u)   (u = wall or inlet)
 *   PRESSURE     f_i(x) = -f*_opp(i)(x) + feq_i + feq_opp(i), the model's
 *                equilibrium at density 1 + face_drho and the node's own
 *                velocity (of its state before the step): the fixed-pressure
 *                outflow of the paper's set-up (Section 3), anti-bounce-back
 *   FREESLIP     f_i(x) = f*_k(x - e_i with the crossed coordinates kept),
 *                k = i with the components normal to the crossed FREESLIP
 *                faces reversed (specular reflection half-way, the
 *                free-slip top of the paper's tank, Section 3)
 *   OUTFLOW      f_i(x) = f*_i(x - e_i with the z coordinate kept)
 *   face_drho  density deviation rho - 1 of LBM_PRESSURE faces (finite and
 *              above -1, else LBM_EINVAL; ignored for other faces).
 * Where a source lies beyond several faces, WALL wins over INLET over
 * PRESSURE over FREESLIP over OUTFLOW. The inlet buffers must stay valid
 * while the lattice steps. Lattices with FREESLIP or PRESSURE faces have no
 * adjoint (lbm_step_record and lbm_adjoint_step refuse them).
 */
typedef struct lbm_boundaries {
  int32_t face_type[6];
  double face_u[6][3];
  const void* inlet_u;
  int32_t inlet_dtype;
  int32_t reserved0;
  const uint8_t* inlet_mask;
  double inlet_amp;
  uint64_t seed;
  double face_drho[6];
} lbm_boundaries;

/* Validate cfg and create a handle (host memory only). On error *out is
 * left untouched. Limits: fewer than 2^31 nodes, nz <= 65535, and one
 * population's storage (nodes x element size) below 4 GiB: 537 M nodes in
 * FP64, 1.07 G in FP32 (the kernels address a population with 32-bit byte
 * offsets).
 *
 * Tracing: with the environment variable LBM_TRACE=1 at creation (here and
 * in lbm_refined_create), the handle times each step-kernel launch (and the
 * link, reduction, adjoint and refinement-interface launches) with HIP events
 * on the stream it runs on, and lbm_destroy / lbm_refined_destroy print per
 * kernel the calls, total, mean, minimum and maximum time to stderr. The
 * events are resolved in batches of 1024 launches (the host waits for that
 * batch); without LBM_TRACE nothing is recorded. Not an operation of the
 * paper. */
int lbm_create_lattice(const lbm_config* cfg, lbm_lattice** out);

/* Bytes of device memory the lattice needs (populations, the outflow ghost
 * plane, reduction partials), 256-byte aligned. */
int lbm_required_bytes(const lbm_lattice* lat, size_t* bytes);

/* Hand over a device block of at least lbm_required_bytes bytes, 256-byte
 * aligned. It must outlive the lattice (or the next bind). Resets the
 * time to 0 and the populations' contents are undefined until
 * lbm_init_equilibrium or lbm_set_populations. */
int lbm_bind_memory(lbm_lattice* lat, void* dev, size_t bytes);

/* Set the boundary description (default: all periodic). Host struct; the
 * device buffers it names are used, not copied. Only valid at an even
 * number of steps since the last set/init/load (LBM_ESTATE otherwise). */
int lbm_set_boundaries(lbm_lattice* lat, const lbm_boundaries* bc);

/* Populations := the model's equilibrium for fields drho (device, rho - 1,
 * nx*ny*nz) and u (device, [3][N]) of dtype LBM_DTYPE_F64/F32: Eq. (2) for
 * MRT, the product equilibrium with the Table 2 central moments for FCLB.
 * Sets the time to t0. */
int lbm_init_equilibrium(lbm_lattice* lat, const void* drho, const void* u,
                         int dtype, int64_t t0);

/* Populations := f (device, [Q][N] deviations f_i - w_i, ABI order, dtype
 * LBM_DTYPE_F64/F32), rounded to the storage type. Sets the time to t0. */
int lbm_set_populations(lbm_lattice* lat, const void* f, int dtype, int64_t t0);

/* f (device, [Q][N]) := current pre-collision populations (deviations, ABI
 * order), whatever the in-place streaming parity. */
int lbm_get_populations(lbm_lattice* lat, void* f, int dtype);

/* Interior solid nodes (a node-type field). solid: device, N bytes
 * ([nz][ny][nx]), nonzero = solid. masks: device work buffer of N uint32
 * owned by the caller, filled here with each node's solid-neighbour mask and
 * read by every later step: it must stay allocated and unchanged until the
 * solids are cleared (solid = NULL), lbm_set_boundaries is called (which
 * clears them) or the lattice is destroyed. A population whose pull source
 * is a solid node bounces back off a wall at rest halfway between the nodes
 * (the rule of a WALL face with zero velocity). Solid nodes take no part in the flow;
 * their populations are unspecified, lbm_get_populations returns zeros and
 * lbm_get_macroscopic the rest state (rho = 1, u = 0) there, and the
 * reductions, statistics and probe count them as rest. Steps then run the
 * general boundary kernel on every row. Blocking (validation).
 * Errors: LBM_EINVAL (masks NULL while solid is given; a solid node on an
 * OUTFLOW face, whose zero-gradient copy would read it: the solids are then
 * left cleared), LBM_EUNBOUND, LBM_ESTATE (odd in-place parity). The adjoint
 * calls (lbm_step_record, lbm_adjoint_step) refuse a lattice with solids. */
int lbm_set_solids(lbm_lattice* lat, const uint8_t* solid, uint32_t* masks);

/* Curved no-slip walls (the second-order interpolated walls of the paper's
 * nozzle, Section 3): Bouzidi's linear interpolated bounce-back on links from
 * fluid nodes to the solid nodes set by lbm_set_solids. For a link from fluid
 * node x towards the solid x + e_k whose wall lies at the fraction q of the
 * link, with i = opp(k) the returning direction:
 *   q <  1/2:  f_i(x) = 2q f*_k(x) + (1 - 2q) f*_k(x - e_k)
 *   q >= 1/2:  f_i(x) = f*_k(x) / (2q) + (2q - 1)/(2q) f*_i(x)
 * replacing the halfway value f*_k(x). Where x - e_k is not a fluid node
 * inside the domain (solid, or beyond a non-periodic face), the halfway
 * value stays.
 *   nodes  device int32 [n]: linear node indices x + nx (y + ny z) of the
 *          fluid nodes that have links, each at most once (a repeated node
 *          gives unspecified results).
 *   q      device float [n][Q]: q[j][k] is the wall distance of the link of
 *          nodes[j] in direction k (ABI order); entries outside (0, 1], or
 *          in a direction whose neighbour is not solid, are ignored (q = 1/2
 *          is the halfway rule itself).
 * Both buffers are owned by the caller and read by every later step: they
 * must stay allocated and unchanged until the links are cleared (n = 0),
 * lbm_set_solids or lbm_set_boundaries is called (both clear them) or the
 * lattice is destroyed. Indices outside [0, N) and solid nodes are skipped.
 * Each step then runs one extra kernel over the n listed nodes.
 * Errors: LBM_EINVAL (n < 0 or n >= 2^31, n > 0 with NULL buffers or no
 * solids set), LBM_EUNBOUND, LBM_ESTATE (odd in-place parity). */
int lbm_set_links(lbm_lattice* lat, const int32_t* nodes, const float* q, int64_t n);

/* Advance n >= 0 collide-and-stream steps (asynchronous, except for the
 * checks that lbm_set_check asks for, which block and may stop the steps
 * early with LBM_ENONFINITE or LBM_EMASS). */
int lbm_step(lbm_lattice* lat, int64_t n);

/* rho (device, N) and u (device, [3][N]) of the current state: MRT
 * Eqs. (3)-(5) with rho0 = 1 (u = j), FCLB Eqs. (6)-(8) (u = j / rho).
 * rho_mode LBM_RHO_FULL writes rho, LBM_RHO_DEVIATION writes rho - 1.
 * Either pointer may be NULL. */
int lbm_get_macroscopic(lbm_lattice* lat, void* rho, void* u, int dtype,
                        int rho_mode);

/* Blocking. FP64 sums over all nodes in a fixed order (deterministic):
 * out[0] = sum (rho - 1), out[1..3] = sum j, out[4] = sum |j|^2 / (2 rho)
 * (rho = 1 for MRT). Returns LBM_ENONFINITE if any sum is not finite
 * (out is still written). */
int lbm_reduce(lbm_lattice* lat, double out[5]);

/* Health check inside lbm_step (the global conservation of Section 2's
 * collisions: mass is a collision invariant, so on a closed or periodic
 * lattice the mass deviation changes only by rounding). With every > 0,
 * after each step whose new step count is a multiple of `every`, lbm_step
 * runs the FP64 sums of lbm_reduce (one extra read of the populations,
 * blocking) and stops, returning LBM_ENONFINITE if a sum is not finite, or
 * LBM_EMASS if mass_tol >= 0 and |sum(rho - 1) - M0| > mass_tol, M0 being
 * the sum when the check was set (every > 0 checks the current state at
 * once, blocking). The steps before
 * the failing check stand (lbm_get_time tells how many ran). mass_tol < 0
 * checks finiteness only (open boundaries change the mass); every = 0 turns
 * the check off. Errors: LBM_EINVAL (every < 0, NaN mass_tol), LBM_EUNBOUND,
 * LBM_ENONFINITE if the current state already has a non-finite sum (the
 * check stays off). */
int lbm_set_check(lbm_lattice* lat, int64_t every, double mass_tol);

/* For callers that cannot allocate device memory or synchronise (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the sums of lbm_reduce written to the caller's DEVICE buffer out[5]
 * (FP64), stream-ordered on the lattice's stream, no host copy and no
 * synchronisation; the caller checks finiteness. The partial sums live in a
 * library-owned static device array (16384 rows of five doubles, about
 * 640 KiB per device, held until the process ends): z planes fold into the
 * blocks of one x-y plane, so the summation order differs from lbm_reduce's
 * (equal up to FP64 rounding). Nothing is allocated. Returns LBM_EINVAL if
 * an x-y plane needs more than 16384 blocks of 256 nodes
 * (ceil(nx / bx) * ceil(ny / by), bx = min(nx, 256), by = 256 / bx).
 * Every call on one device shares the array: calls that overlap on one
 * device (different streams, threads or lattices) race. */
int lbm_reduce_static(lbm_lattice* lat, double* out);

/* Time averages of the velocity: the jet statistics of Section 3 (mean
 * velocity; turbulent intensity, Eq. (25)). The caller owns an FP64 device
 * buffer sums of 6 x N values ([6][N]: running sums of u_x, u_y, u_z and of
 * u_x^2, u_y^2, u_z^2), zeroes it to start and counts the calls.
 * lbm_stats_accumulate adds the velocity of the current state (u as in
 * lbm_get_macroscopic). Asynchronous on the lattice's stream.
 * Errors: LBM_EINVAL (null pointer), LBM_EUNBOUND. */
int lbm_stats_accumulate(lbm_lattice* lat, double* sums);

/* Spreading of the jet (Section 3: the width of Eq. (23), the profile of
 * Eq. (24)) from a time-averaged velocity, on every cross-section normal to
 * the jet axis. mean: device [3][nz][ny][nx] of dtype (LBM_DTYPE_F64/F32),
 * e.g. the mean of lbm_stats_finalize. The streamwise component is
 * interpolated bilinearly in the section's coordinates (a, b) (the two other
 * axes in increasing order); u_m is its value at the jet centre (c0, c1).
 * Rays leave the centre at the angles 2 pi j / ndir (j < ndir, from a
 * towards b), sampled at r_k = k dr (k < nr) while the sample lies within
 * the section's nodes; a ray's radius r_e is the first point where u falls
 * to 0.368 u_m (half the spreading width), interpolated linearly between
 * the samples around it. Outputs (device, FP64, n_p = the axis extent):
 *   um    [n_p]     u_m of each section;
 *   re    [3][n_p]  minimum, maximum and mean of r_e over the rays that
 *                   reach it (NaN where none does);
 *   prof  [n_p][nr] (may be NULL) mean of u(r_k) / u_m over the rays whose
 *                   sample k lies within the section (NaN where none).
 * Meaningful for u_m > 0 (a jet). Asynchronous on the lattice's stream; the
 * lattice's populations are not read. Errors: LBM_EINVAL (null mean, um or
 * re; bad dtype or axis; ndir outside [1, 65536], nr outside [2, 65536],
 * dr not positive; a section narrower than 2 nodes; the centre outside
 * [0, n_a - 1] x [0, n_b - 1]). */
int lbm_jet_profile(const lbm_lattice* lat, const void* mean, int dtype, int axis, double c0,
                    double c1, int ndir, double dr, int nr, double* um, double* re,
                    double* prof);

/* The jet laws of Section 3 fitted to an lbm_jet_profile result (um [np],
 * re [3][np], prof [np][nr], all device FP64, with its dr) over the
 * sections p0 <= p < p1 downstream of the nozzle exit at axis coordinate x0
 * (distance x = p - x0 > 0; sections with NaN inputs are skipped), for the
 * inflow speed u0 and nozzle diameter d (lattice units):
 *   out[0]  k_par, least squares of u_m = u0 k_par d / x      (Eq. (22))
 *   out[1]  k_perp, least squares of b_g = k_perp x, b_g the mean r_e
 *           (the radius of 0.368 u_m)                          (Eq. (23))
 *   out[2]  root mean square of prof - 0.938 exp(-0.944 (r / r_e)^2)
 *           over the samples r = k dr <= 2 r_e                 (Eq. (24))
 *   out[3]  the number of profile samples in out[2]
 * NaN where nothing enters a fit. out: device, 4 doubles. Asynchronous on
 * the lattice's stream. Errors: LBM_EINVAL (null pointers; np or nr < 1;
 * not 0 <= p0 < p1 <= np; dr or d not positive; u0 zero; non-finite x0). */
int lbm_jet_fit(const lbm_lattice* lat, const double* um, const double* re, const double* prof,
                int np, int nr, double dr, double x0, double u0, double d, int p0, int p1,
                double* out);

/* Averages of count >= 1 accumulated states, in dtype (LBM_DTYPE_F64/F32):
 * mean ([3][N]) = sums / count; rms ([3][N]) = sqrt(<u_a^2> - <u_a>^2), the
 * root-mean-square fluctuation (0 where rounding makes the difference
 * negative); ti (N values, may be NULL) = the turbulent intensity of
 * Eq. (25): the rms of the streamwise component over the mean streamwise
 * velocity at the jet-axis point of the node's cross-section. axis: the
 * streamwise direction (0 x, 1 y, 2 z); (p0, p1): the jet-axis point in the
 * two other coordinates in increasing order (checked only if ti is given).
 * Asynchronous. Errors: LBM_EINVAL (null sums/mean/rms, count < 1, bad dtype,
 * axis or axis point). */
int lbm_stats_finalize(const lbm_lattice* lat, const double* sums, int64_t count, void* mean,
                       void* rms, void* ti, int dtype, int axis, int p0, int p1);

/* Size in bytes of a state snapshot (populations + outflow ghost plane). */
int lbm_state_bytes(const lbm_lattice* lat, size_t* bytes);

/* Copy the state into / out of a device buffer of lbm_state_bytes bytes
 * (asynchronous device-to-device copy). save returns the time and the
 * in-place streaming parity; load takes them back. */
int lbm_save_state(lbm_lattice* lat, void* dev, size_t bytes, int64_t* t,
                   int32_t* parity);
int lbm_load_state(lbm_lattice* lat, const void* dev, size_t bytes, int64_t t,
                   int32_t parity);

/* Current time (number of steps since time 0 as set by init/set/load). */
int lbm_get_time(const lbm_lattice* lat, int64_t* t);

/* Replace the stream used by later asynchronous calls. */
int lbm_set_stream(lbm_lattice* lat, void* stream);

/* Destroy the handle (device memory stays with the caller). NULL is OK. */
int lbm_destroy(lbm_lattice* lat);

/* Static message for a status code; for LBM_EHIP the HIP error text of the
 * last failure on this thread. */
const char* lbm_strerror(int status);

/* Device-to-device copy of n bytes through a plain vectorised kernel on the
 * given stream: the achievable-bandwidth probe used for roofline scaling.
 * Both buffers device, 16-byte aligned, non-overlapping. */
int lbm_stream_copy(void* dst, const void* src, size_t n, void* stream);


/* ======================================================================
 * Discrete adjoint of the D3Q27 FCLB and D3Q19 MRT-LES collide-and-stream
 * steps (the collisions of Section 2, Eq. (12) with the Smagorinsky
 * relaxation time of Eqs. (16)-(21) for MRT-LES, with the streaming and
 * boundary rules above). Not an operation of the paper: it differentiates
 * the paper's uniform updates so that gradients of a flow objective with
 * respect to the inlet velocity can be taken through many steps. Where the
 * strain magnitude Q of Eq. (19) is zero its derivative is taken as 0.
 *
 * One step maps the pre-collision state f_t to f_{t+1} = S(C(f_t); u_in).
 * For an objective J(f_T), lambda_T = dJ/df_T and
 *   lambda_t = J_C(f_t)^T S^T lambda_{t+1},
 * and the gradient of J with respect to the inlet velocity collects, at each
 * inlet-face node and each step, 6 w_i e_i lambda_{t+1,i} over the
 * directions i that bounce back through the inlet face.
 *
 * Layout of f_t and lambda: natural pre-collision order [Q][nz][ny][nx] in
 * the velocity order of Section 2, as returned by lbm_get_populations (full
 * deviations f_i - w_i for f_t). dtype is the adjoint's arithmetic and
 * storage type: LBM_DTYPE_F64 or LBM_DTYPE_F32, the same for f_t and both
 * lambda arrays. All buffers are caller-owned device memory; work is queued
 * on the lattice's stream and the lattice's own state is not touched.
 * ====================================================================== */

/* Probe objective of the current pre-collision state: J = mean over the
 * box lo <= (x, y, z) < hi of |j|^2 / (2 rho), with rho = 1 + sum f for the
 * FCLB model and rho = 1 for the incompressible MRT model. If lambda is not
 * NULL it receives dJ/df (zero outside the box) in dtype. Blocking: J is
 * returned on the host. LBM_EINVAL for an empty or out-of-range box. */
int lbm_probe_ke(lbm_lattice* lat, const int32_t lo[3], const int32_t hi[3], void* lambda,
                 int dtype, double* J);

/* One FCLB or MRT-LES step (as lbm_step with n = 1) that also writes the
 * natural pre-collision state it collides, i.e. what lbm_get_populations
 * would have returned before the step, into rec ([Q][nz][ny][nx], device).
 * dtype must be the adjoint's type: LBM_DTYPE_F64 for FP64 storage,
 * LBM_DTYPE_F32 for FP32 storage; FP16 storage, the CLB model, solid nodes
 * and free-slip or pressure faces give LBM_EINVAL. At inlet and
 * wall nodes of FP32 storage the bounce-back term is added in FP32, as the
 * step computes it (lbm_get_populations adds it in FP64). Asynchronous. */
int lbm_step_record(lbm_lattice* lat, void* rec, int dtype);

/* One adjoint step: lambda = J_C(f_t)^T S^T lambda_next for the lattice's
 * configuration and boundaries (FCLB or MRT-LES, without solid nodes,
 * free-slip or pressure faces, else LBM_EINVAL). grad_inlet,
 * if not NULL, is a device double array [3][nb][na] laid out like the
 * inlet velocity field of lbm_boundaries, to which this step's inlet terms
 * are added. lambda must not alias lambda_next or f_t; one population of an
 * adjoint array (nodes x element size) must stay below 4 GiB, else
 * LBM_EINVAL. Asynchronous. */
int lbm_adjoint_step(lbm_lattice* lat, const void* f_t, const void* lambda_next, void* lambda,
                     int dtype, double* grad_inlet);

/* ======================================================================
 * Nested time refinement on a hierarchical block grid (the block grid with
 * nested time steps of Section 1 and the refinement levels of the numerical
 * set-up in Section 3; interface interpolation and rescaling after Yu et
 * al., cited there without formulas).
 *
 * Level 0 is the lattice cfg->nx x ny x nz (lattice viscosity cfg->nu),
 * divided into blocks of block^3 nodes. A level map gives, per level-0
 * block, the finest level that covers it; R_l, the region of level l, is
 * the union of the blocks whose entry is >= l. Level l has 2^l times the
 * resolution in space and time (the same velocity scale: constant CFL
 * number), lattice viscosity 2^l nu (tau_l - 1/2 = 2^l (tau_0 - 1/2)); the
 * Smagorinsky constant acts in each level's own lattice units. Nesting is
 * cell-centred: level-(l+1) node j lies at level-l coordinate j/2 - 1/4 (a
 * node's cell holds the children 2i and 2i+1 on each axis), so the halfway
 * walls, inlets and faces of all levels coincide.
 *
 * One lbm_refined_step advances one level-0 step: level l steps 2^l times,
 * recursively (each level steps once, then its child level twice). Every
 * level holds post-collision populations (deviations, ABI order) in a box:
 * R_l plus the layer of ghost nodes around it, with its x origin and row
 * pitch rounded to multiples of 64 nodes (extra nodes are unused).
 * Interface per parent step t:
 *   child ghosts, first substep:  rescale(G(t)),
 *   child ghosts, second substep: rescale(-1/8 G(t-1) + 3/4 G(t) + 3/8
 *     G(t+1)) (1/2 G(t) + 1/2 G(t+1) on the first step after a state
 *     change), G = the parent state interpolated at the ghosts (tensor
 *     4-point cubic Lagrange at the child positions; windows kept inside
 *     non-periodic domains);
 *   rescale = the model's equilibrium plus the non-equilibrium part scaled
 *     by Chapman-Enskog: FCLB/CLB by r = (tau_f - 1)/(2 (tau_c - 1)); MRT
 *     per moment group (tau = 1/s, same non-shear rates on both levels:
 *     1/2, or 0 for rate 1), the shear group with the total relaxation
 *     times of Eq. (20) (tau_c,tot recovered from the interpolated state's
 *     post-collision traceless stress, tau_f,tot = tau0_f + (tau_c,tot -
 *     tau0_c)/2);
 *   covered parent nodes (inside R_{l+1}, read by no ghost interpolation)
 *     that a parent fluid or band node pulls from take the mean of their
 *     eight children, rescaled back, after the two child substeps (no other
 *     covered node is ever read; its slots are left as they are).
 * Node types (lbm_refined_types): 0 unused, 1 fluid, 2 band (inside the
 * next level's region but updated on this level, read by its ghost
 * interpolation), 3 covered, 4 ghost, 5 solid.
 * ====================================================================== */
typedef struct lbm_refined lbm_refined;

/* nlevels in [1, 8]; level_map: host uint8 [nz/block][ny/block][nx/block],
 * entries < nlevels (copied); block >= 2 divides nx, ny, nz (block >= 3
 * with three or more levels). Nesting: every block whose entry is m >= 2
 * has its 26 neighbour blocks (periodic axes wrapping) at m - 1 or more;
 * on a periodic axis each region either spans the axis or keeps off both
 * ends; non-periodic axes need 4 or more nodes. tau = 3 nu 2^l + 1/2 must
 * differ from 1 on every level of a refined lattice (the rescale factor and
 * its inverse must exist) and omega < 2. A configuration that is valid only
 * with non-periodic faces is created and needs lbm_refined_set_boundaries
 * before binding. */
int lbm_refined_create(const lbm_config* cfg, int32_t block, int32_t nlevels,
                       const uint8_t* level_map, lbm_refined** out);

/* Box of level l: origin lo (level coordinates), extent dims (dims[0] is the
 * row pitch, a multiple of 64); counts = {fluid, band, covered, ghost,
 * solid} nodes. LBM_ESTATE while the configuration waits for boundaries. */
int lbm_refined_geometry(const lbm_refined* r, int32_t level, int32_t lo[3], int32_t dims[3],
                         int64_t counts[5]);

/* Node types of level l's box (host uint8 [dims z][y][x], codes above). */
int lbm_refined_types(const lbm_refined* r, int32_t level, uint8_t* types);

/* Bytes of device memory (three state arrays per level, node types, tile lists,
 * ghost lists and interface history, solid lists, reduction scratch). Valid
 * after the last set_boundaries / set_solids / set_links. */
int lbm_refined_required_bytes(const lbm_refined* r, size_t* bytes);

/* Hand over the device block (256-byte aligned) and upload the geometry;
 * blocking. Resets the time to 0. LBM_ESTATE if the configuration still
 * waits for boundaries. */
int lbm_refined_bind_memory(lbm_refined* r, void* dev, size_t bytes);

/* Boundary description of the domain (as lbm_set_boundaries, applied on
 * every level; LBM_FREESLIP and LBM_PRESSURE faces included; outflow may be
 * any face). With an inlet face each level l >= 1 needs its own inlet arrays
 * at its resolution: level_inlet_u[l] ([3][2^l nb][2^l na], bc->inlet_dtype)
 * and, if bc->inlet_mask is given, level_inlet_mask[l] ([2^l nb][2^l na]);
 * both host arrays of nlevels device pointers, entry 0 unused (level 0 takes
 * bc's own). Level l draws its perturbation with seed + l and its own step
 * index. Must precede lbm_refined_bind_memory (LBM_ESTATE after it); the
 * device buffers must stay valid while the lattice steps. */
int lbm_refined_set_boundaries(lbm_refined* r, const lbm_boundaries* bc,
                               const void* const* level_inlet_u,
                               const uint8_t* const* level_inlet_mask);

/* Interior solid nodes of level l (the nozzle of the paper's set-up,
 * Section 3): host uint8 over the level's box ([dims z][y][x], copied),
 * nonzero = solid; NULL clears. Populations whose source is solid bounce
 * back halfway (a wall at rest) or along curved links (lbm_refined_set_links).
 * Solids keep off the interfaces: no solid ghost or band node, no solid
 * next to a ghost, and no solid child under a covered node that a parent-
 * updated node reads (LBM_EINVAL, solids unchanged). Clears the level's
 * links. Must precede lbm_refined_bind_memory (LBM_ESTATE after it). */
int lbm_refined_set_solids(lbm_refined* r, int32_t level, const uint8_t* solid);

/* Curved walls on level l (Bouzidi's linear interpolated bounce-back, the
 * rule of lbm_set_links): host arrays, copied: nodes [n] box indices of fluid
 * nodes, q [n][Q] wall distances (entries outside (0, 1], or where the
 * neighbour is not solid, ignored; where the node behind along the link is
 * solid or beyond a face the halfway rule stays). Needs solids on that
 * level (LBM_EINVAL otherwise); must precede lbm_refined_bind_memory. */
int lbm_refined_set_links(lbm_refined* r, int32_t level, const int32_t* nodes, const float* q,
                          int64_t n);

/* Equilibrium state of one level's box (fields [dims] and [3][dims]), as
 * lbm_init_equilibrium. Sets the time; the interface history restarts. */
int lbm_refined_init_equilibrium(lbm_refined* r, int level, const void* drho, const void* u,
                                 int dtype, int64_t t0);

/* Post-collision populations of one level's box, [Q][dims] (set / get).
 * Ghost nodes hold interface values prepared for the next substep, not
 * state; solid nodes hold values of the solid pre-pass; covered nodes over
 * a finer level's covered nodes are not updated. A set restarts the
 * interface history and sets the time. */
int lbm_refined_set_populations(lbm_refined* r, int level, const void* f, int dtype,
                                int64_t t0);
int lbm_refined_get_populations(lbm_refined* r, int level, void* f, int dtype);

/* Advance n level-0 steps (asynchronous, on the lattice's stream). */
int lbm_refined_step(lbm_refined* r, int64_t n);

/* rho and u of one level's box (as lbm_get_macroscopic). */
int lbm_refined_get_macroscopic(lbm_refined* r, int level, void* rho, void* u, int dtype,
                                int rho_mode);

/* Blocking FP64 sums over the domain: the fluid nodes of every level that
 * no finer level covers, weighted by their volume 8^-l in level-0 cells. */
int lbm_refined_reduce(lbm_refined* r, double out[5]);

int lbm_refined_get_time(const lbm_refined* r, int64_t* t);
int lbm_refined_set_stream(lbm_refined* r, void* stream);
int lbm_refined_destroy(lbm_refined* r);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
