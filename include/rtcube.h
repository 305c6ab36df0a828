/*
 * rtcube.h -- C ABI of the MI355X line radiative-transfer renderer.
 *
 * The library renders spectral data cubes of LTE molecular line emission from
 * an azimuthally and mirror-symmetric protoplanetary disk, and differentiates
 * them.  Physics (Methods, "Line Radiative Transfer"): the formal solution of
 * Eq. rt-int with the optical depth of Eq. optical_depth, LTE emissivity j and
 * extinction beta from Boltzmann level populations, a Gaussian Doppler profile
 * shifted by the projected velocity and broadened by thermal + turbulent
 * motions.  Disk model (Methods, "Parametric Disk Modeling"): H2 density,
 * temperature and azimuthal velocity on an (r, z/r) grid, with the CO layer
 * between a freeze-out and a photodissociation surface (Eq. co_layer).
 *
 * Discretisation (identical in every entry point):
 *   - grid nodes r_i = r_min (r_max/r_min)^(i/(nr-1)), (z/r)_j = zr_max j/(nz-1);
 *     fields are bilinear in (ln r, z/r) index space, clamped to the edge, and
 *     the density fades linearly to zero one cell beyond the last node;
 *   - CO abundance x_co times a logistic mask sigma((z_up-|z|)/w) sigma((|z|-z_lo)/w),
 *     w = mask_width * r * d(z/r), with z_lo / z_up linear in the radial index;
 *   - orthographic camera: pixel centres ((p+1/2-nx/2) d, (q+1/2-ny/2) d),
 *     d = fov/nx, rotated by the position angle; ray direction
 *     (0, sin i, -cos i); gas rotates counter-clockwise about +z;
 *   - each ray's chord through the cylinder r <= r_max e^dln, |z| <= (zr_max +
 *     d(z/r)) r_max e^dln is cut into nsamp equal segments; each segment holds
 *     the fields of its midpoint and contributes S (1 - e^-dtau) attenuated by
 *     everything in front of it (no background);
 *   - channels are velocities v_c [km/s] (radio convention); the profile of a
 *     channel depends on (v_los - v_c) / alpha only.
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers into caller-owned HIP memory unless
 *     marked [host].  Layouts: fields [nr][nz] (z/r index fastest), surfaces
 *     [nr], cubes [nch][ny][nx] (x fastest), all float32.
 *   - Arguments are validated on the host only; device data is never read
 *     for validation, so NaNs in inputs propagate to outputs.
 *   - Work is enqueued on the given HIP stream (a hipStream_t passed as
 *     void*, NULL = the null stream) and the call returns without waiting;
 *     buffers must stay valid until that stream work has completed.
 *   - Outputs are written only when the call returns RT_OK; gradients are
 *     overwritten, not accumulated.
 *   - On any non-OK status rt_last_error() returns a message (thread-local).
 */
#ifndef RTCUBE_H
#define RTCUBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_ABI_VERSION 1
#define RT_MAX_CHANNELS 4096     /* per call; larger cubes are several calls */

typedef enum {
    RT_OK = 0,
    RT_PENDING = 1,       /* server ticket not finished yet */
    RT_EINVAL = -1,       /* invalid argument (see rt_last_error) */
    RT_ENOMEM = -2,       /* device allocation failed */
    RT_EDEVICE = -3,      /* a HIP call or kernel launch failed */
    RT_EAGAIN = -4,       /* server pending queue full: retry later */
    RT_ECANCELED = -5,    /* request cancelled before it ran */
    RT_ETOOBIG = -6,      /* request footprint exceeds the server's HBM budget */
    RT_ENOTFOUND = -7     /* unknown server ticket */
} rt_status;

/* (r, z/r) node grid: nr, nz >= 2; 0 < r_min_au < r_max_au; zr_max > 0. */
typedef struct {
    int32_t nr, nz;
    double r_min_au, r_max_au, zr_max;
} rt_grid;

/* Disk fields.  ln_nh2: natural log of n_H2 [cm^-3]; temp_k: gas temperature
 * [K] (must be > 0); vphi_kms: azimuthal velocity [km/s]; z_lo_au / z_up_au:
 * lower (freeze-out) and upper (photodissociation) CO surface heights per
 * radial node [au].  x_co: CO abundance inside the layer; mask_width: mask
 * width in units of r d(z/r) (> 0); v_turb: turbulent Mach number. */
typedef struct {
    const float *ln_nh2, *temp_k, *vphi_kms;   /* [nr][nz] */
    const float *z_lo_au, *z_up_au;            /* [nr] */
    double x_co, mask_width, v_turb;
} rt_fields;

/* One line transition in LTE.  lev_e_k / lev_g: [host] energies [K] and
 * degeneracies of the levels summed in the partition function (copied during
 * the call; the partition function is tabulated for 0.1 K <= T <= 1e4 K and
 * clamped outside).  m_mol_amu: mean molecular mass of the gas [amu]. */
typedef struct {
    double nu0_hz, a_ul, g_u, g_l, e_u_k, e_l_k, m_co_amu, m_mol_amu;
    int32_t nlev;
    const double *lev_e_k, *lev_g;
} rt_line;

/* Orthographic camera: nx x ny pixels over fov_au along x (square pixels);
 * inclination 0..90 deg; position angle rotates the image plane. */
typedef struct {
    int32_t nx, ny;
    double fov_au, incl_deg, pa_deg, dist_pc;
} rt_camera;

/* Spectral axis: nch channel velocities [km/s] ([host], copied during the
 * call) and the systemic velocity added to every line-of-sight velocity. */
typedef struct {
    int32_t nch;
    const double *v_kms;
    double v_sys_kms;
} rt_spectral;

/* Restoring beam of an image (see rt_beam_convolve): FWHM bmaj_px >= bmin_px
 * in pixels, major axis at bpa_deg from +y towards -x. */
#define RT_BEAM_MAX_RADIUS 24    /* R <= 24 pixels: bmaj_px <= 18.8 */
typedef struct {
    double bmaj_px, bmin_px, bpa_deg;
} rt_beam;

/* Neural CO layer (optional): 16 Fourier frequencies 2^(3k/15) on the two
 * normalised grid coordinates, 4 SiLU hidden layers of width 128, 3 outputs
 * giving z_up = zr_max r sigma(o0), z_lo = zr_max r sigma(o1) and
 * T <- T exp(0.5 tanh(o2)).  weights: float32, per layer W [out][in] then
 * b [out].  precision: RT_MLP_BF16 (BF16 matrix cores, FP32 accumulation) or
 * RT_MLP_FP32. */
enum { RT_MLP_FP32 = 0, RT_MLP_BF16 = 1 };
#define RT_MLP_PARAMS 58243
typedef struct {
    const float *weights;
    int32_t precision;
} rt_mlp;

typedef struct {
    rt_grid grid;
    rt_fields f;
    rt_line line;
    rt_camera cam;
    rt_spectral spec;
    int32_t nsamp;             /* samples per ray, >= 1 */
    double intensity_scale;    /* output = scale * I_nu [erg s^-1 cm^-2 Hz^-1 sr^-1] */
    const rt_mlp *mlp;         /* NULL: surfaces and temperature from the grid */
} rt_problem;

/* Gradient outputs, each NULL when not requested. */
typedef struct {
    float *d_ln_nh2, *d_temp_k, *d_vphi_kms;   /* [nr][nz] */
    float *d_z_lo_au, *d_z_up_au;              /* [nr] */
    float *d_mlp;                              /* [RT_MLP_PARAMS] */
} rt_grads;

/* Render the cube [nch][ny][nx] of problem p. */
rt_status rt_render_cube(const rt_problem *p, float *cube, void *stream);

/* Vector-Jacobian product of rt_render_cube: given dL/dcube [nch][ny][nx],
 * write the requested gradients of L w.r.t. the fields, surfaces and network
 * weights.  cube_opt (may be NULL) receives the forward cube.  Nothing per
 * sample and channel is stored: the reverse sweep recomputes every sample's
 * line terms from a per-sample tape and rebuilds its transmission from the
 * ray's total optical depth (the single checkpoint per ray and channel) minus
 * the depth behind it, or, with RT_OPT_CKPT_SEGMENT, from transmission
 * checkpoints every few samples.  Gradients use atomics, so their last bits
 * may vary from run to run.  With the network (p->mlp) a call takes at most
 * 256 channels and fewer than 2^32 - 1 pixel-samples (nx ny nsamp);
 * RT_EINVAL otherwise. */
rt_status rt_render_cube_adjoint(const rt_problem *p, const float *dl_dcube, const rt_grads *g,
                                 float *cube_opt, void *stream);

/* Forward + L2 loss + adjoint in one pass (the fitting step of Fig.
 * radjax_pipeline with an L2 pixel loss, Methods > Neural temperature
 * recovery): L = sum (cube - target)^2 over [nch][ny][nx].  Writes the cube
 * (device, required), the requested gradients of L as rt_render_cube_adjoint
 * does for dL/dcube = 2 (cube - target), and, if loss != NULL, L to *loss
 * (device pointer to one double).  The reverse march forms dL/dcube from its
 * own forward sweep, so no separate forward render is run.  target: device,
 * [nch][ny][nx].  At most 256 channels per call. */
rt_status rt_render_cube_l2_adjoint(const rt_problem *p, const float *target, const rt_grads *g, float *cube,
                                    double *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * as rt_render_cube_l2_adjoint for grid fields (no network), but it calls no
 * allocator.  The library's scratch for the call (partition-function table,
 * gradient accumulators, the sample tape and cotangents of one band of
 * image rows; the image is processed band by band) lives in one fixed device
 * array of rt_noalloc_scratch_bytes() bytes (256 MiB) per GPU, held until
 * the process ends.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller.  Each call clears what must start at zero.
 * Returns RT_ETOOBIG, before any GPU work, when the table, the accumulators
 * and one row of pixels do not fit the array; RT_EINVAL for a network
 * problem, more than 256 channels or NULL target / cube / grads. */
rt_status rt_render_cube_l2_adjoint_noalloc(const rt_problem *p, const float *target, const rt_grads *g,
                                            float *cube, double *loss, void *stream);
/* Size in bytes of the fixed array rt_render_cube_l2_adjoint_noalloc uses. */
uint64_t rt_noalloc_scratch_bytes(void);

/* Work accounting of rt_render_cube on problem p (Methods > Line RT: a ray
 * has samples only over its chord through the grid's bounding cylinder):
 * counts[0] = rays that cross the cylinder (the others have no samples, zero
 * intensity and no work), counts[1] = their pixel-samples, counts[2] = those
 * pixel-samples whose line-centre depth is below the march's thin-sample
 * threshold (taken with the series form of 1 - e^-dtau), counts[3] = those
 * with any opacity (K > 0; a sample with K = 0 changes no channel), counts[4]
 * = those inside the grid's edge taper (the march shades only these in
 * full), the last three -1 for a problem with the network (its shading
 * needs the network's outputs).  counts: [host] int64[5].  mask (device, [ny][nx] bytes, may be
 * NULL) receives 1 for each
 * crossing ray, 0 otherwise.  The march's own ray set-up and shading are
 * used.  Synchronous: returns after the stream's work is done. */
rt_status rt_render_census(const rt_problem *p, uint8_t *mask, int64_t *counts, void *stream);

/* ------------------------------------------------------- derived fields */
/* Fields derived from a temperature grid, as the physics-informed
 * constraints of Methods > Neural temperature recovery derive them (equations
 * of Methods > Parametric disk modeling):
 *   - n_H2 from vertical hydrostatic equilibrium, Eq. gas_density_temp,
 *     integrated up each column from the midplane and normalised so that the
 *     column holds the tapered power-law surface density
 *     Sigma(r) = Sigma0 (r/r_c)^-gamma exp(-(r/r_c)^(2-gamma)),
 *     Sigma0 = M_gas (2 - gamma) / (2 pi r_c^2); n_H2 = rho / (mu m_H);
 *   - the vertical H2 column of Eq. column_density and from it the CO surfaces
 *     of Eq. co_layer: z_up where 0.706 N_H2 = n_dissoc, z_lo where
 *     T = t_freeze;
 *   - v_phi from gravity and the radial pressure gradient,
 *     Eq. gas_velocity_pressure, with P = n_H2 k_B T.
 * Discretisation on the render grid (rt_grid): per radial node, the trapezoid
 * rule on the z/r nodes for the gravity term and the column (the log-T term
 * of the hydrostatic equation exactly); z_up log-linear in N between the last
 * node above the threshold and the next (linear to the top node, where
 * N = 0), -zr_max r when even the midplane is below it; z_lo linear in T
 * between the last cold and the first warm node, -zr_max r for a warm
 * midplane, 2 zr_max r for a column never warm; d ln P / d ln r at fixed
 * height as central differences of ln(n T) along ln r and z/r on the node
 * grid (one-sided at its edges); v_phi = sqrt(max(v^2, 0)).  The outputs are
 * the ln_nh2, vphi_kms, z_lo_au and z_up_au of rt_fields.  Computed in FP32. */
typedef struct {
    rt_grid grid;                        /* nz <= 2048 */
    const float *temp_k;                 /* [nr][nz] device, > 0 */
    double mstar_msun;                   /* stellar mass, >= 0 */
    double mgas_msun, rc_au, gamma;      /* Sigma(r): M_gas > 0, r_c > 0, gamma < 2 */
    double mu;                           /* mean molecular weight, m_mol = mu m_H */
    double t_freeze_k, n_dissoc_cm2;     /* CO-layer thresholds, > 0 */
} rt_derive;

typedef struct {
    float *ln_nh2, *vphi_kms;            /* [nr][nz] device */
    float *z_lo_au, *z_up_au;            /* [nr] device */
} rt_derived;

/* The two-layer temperature of Methods > Parametric disk modeling at every
 * node: T_mid = t_mid0 (r/r_scale)^q, T_atm = t_atm0 (r/r_scale)^q,
 * T = T_atm + (T_mid - T_atm) cos^(2 delta)(pi z / (2 z_q)) below
 * z_q = zq0 (r/r_scale)^1.3 and T_atm above (a single power-law index). */
typedef struct {
    double t_mid0_k, t_atm0_k, q, r_scale_au, zq0_au, delta;
} rt_param_temp;
rt_status rt_parametric_temperature(const rt_grid *grid, const rt_param_temp *pt, float *temp_k, void *stream);

/* Write every field of *out (all four required). */
rt_status rt_derive_fields(const rt_derive *d, const rt_derived *out, void *stream);

/* Vector-Jacobian product of rt_derive_fields: cot holds dL/d(each output)
 * (read only; a NULL member counts as zero); d_temp_k [nr][nz] receives dL/dT
 * through the derived fields (overwritten; the direct temperature gradient of
 * rt_render_cube_adjoint is separate, and the caller adds the two).  The
 * surfaces are differentiated with their bracketing nodes held at those the
 * forward picks at this temperature.  Scratch of 5 nr nz floats is kept with
 * the stream. */
rt_status rt_derive_fields_adjoint(const rt_derive *d, const rt_derived *cot, float *d_temp_k, void *stream);
/* The same, but the product is added to d_temp_k (which holds, say, the
 * render's direct dL/dT), so the two parts of dL/dT of a fit through the
 * derived fields sum on the device. */
rt_status rt_derive_fields_adjoint_add(const rt_derive *d, const rt_derived *cot, float *d_temp_k, void *stream);

/* --------------------------------------------------- neural temperature */
/* The neural temperature field of Methods > Neural temperature recovery on the
 * nodes of the render grid: T = 5 + 395 sigma(o) K, o = MLP(gamma(x_r, x_z)),
 * with the sinusoidal encoding of degree 4 of the normalised node coordinates
 * x_r = i/(nr-1), x_z = j/(nz-1): sin(2^k pi x_r), cos(2^k pi x_r),
 * sin(2^k pi x_z), cos(2^k pi x_z) for k = 0..3 (16 features in that order),
 * then four fully connected layers of 64 units with ReLU and one output.
 * Weights: float32 device array of RT_NT_PARAMS, per layer W [out][in] then
 * b [out].  FP32. */
#define RT_NT_PARAMS 13633

/* temp_k [nr][nz] = T at every node (nr, nz >= 2). */
rt_status rt_neural_temperature(const rt_grid *grid, const float *weights, float *temp_k, void *stream);

/* Vector-Jacobian product: d_weights [RT_NT_PARAMS] = (dT/dweights)^T
 * d_temp_k (overwritten; sums over nodes in a fixed order, so the result is
 * reproducible).  Scratch of about 2100 bytes per node is kept with the
 * stream. */
rt_status rt_neural_temperature_adjoint(const rt_grid *grid, const float *weights, const float *d_temp_k,
                                        float *d_weights, void *stream);

/* Adam (Kingma & Ba) on n float32 parameters in place, with first / second
 * moment buffers m and v (zero before step 1) and step >= 1 the 1-based step
 * count for the bias corrections; the gradient is multiplied by grad_scale
 * first (e.g. 1/sigma^2 turning an L2 gradient into a chi^2 one). */
typedef struct {
    double lr, beta1, beta2, eps, grad_scale;
} rt_adam;
rt_status rt_adam_step(float *params, float *m, float *v, const float *grad, int64_t n, const rt_adam *opt,
                       int64_t step, void *stream);

/* ---------------------------------------------------------------- server */
/* Continuous-batching render server on one GPU.  Requests are admitted in
 * arrival order while their HBM footprint (inputs, outputs and library
 * scratch) fits the budget and a slot is free.  Admitted plain forward
 * requests too small to fill the device alone (fewer pixel x 16-channel
 * lanes than the persistent launch keeps resident) are cut into (tile,
 * channel block) work items that one persistent launch pulls from a device
 * counter; larger forward requests take rt_render_cube's launch, and gradient
 * and neural-layer requests their own sequence of launches, each on a stream
 * of its own; requests that arrive meanwhile start on the next idle stream,
 * so work of different requests overlaps on the device.  A
 * request's forward cube depends only on the request (bitwise the same alone
 * and in any mix) and equals rt_render_cube's to FP32 rounding.  The caller's
 * device buffers must stay valid until the ticket is done or cancelled. */
typedef struct rt_server rt_server;

typedef struct {
    uint64_t hbm_budget_bytes;   /* admission budget for request footprints */
    int32_t max_slots;           /* requests admitted at once (1..1024) */
    int32_t max_pending;         /* queued, not yet admitted (>= 1) */
    int32_t device;              /* HIP device ordinal */
    int32_t streams;             /* launches in flight at once (1..8) */
} rt_server_cfg;

enum { RT_REQ_FWD = 0, RT_REQ_FWD_ADJ = 1, RT_REQ_FWD_LOSS = 2 };
enum { RT_TICKET_QUEUED = 0, RT_TICKET_RUNNING = 1, RT_TICKET_DONE = 2, RT_TICKET_CANCELED = 3,
       RT_TICKET_FAILED = 4 };

/* kind RT_REQ_FWD renders into cube; RT_REQ_FWD_ADJ also takes target
 * [nch][ny][nx] and writes the gradients of L = sum (cube - target)^2 into
 * grads (L itself is reported by rt_poll); RT_REQ_FWD_LOSS renders and
 * reports L without gradients (a likelihood evaluation, e.g. one walker of an
 * ensemble sampler), batched with the other small forwards, L summed on the
 * device in FP64. */
typedef struct {
    rt_problem problem;          /* host copy is taken at submit time */
    int32_t kind;
    float *cube;                 /* device, [nch][ny][nx] */
    const float *target;         /* device, RT_REQ_FWD_ADJ and RT_REQ_FWD_LOSS */
    rt_grads grads;              /* device, RT_REQ_FWD_ADJ only */
    rt_beam beam;                /* RT_REQ_FWD_LOSS only: bmaj_px > 0 convolves the rendered cube with
                                    this beam before the loss (cube then holds the convolved cube);
                                    all zero = no beam */
} rt_request;

typedef struct {
    int32_t state;               /* RT_TICKET_* */
    int32_t status;              /* rt_status of the request */
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;   /* steady-clock stamps */
    double loss;                 /* RT_REQ_FWD_ADJ / RT_REQ_FWD_LOSS: L once done */
    uint64_t ray_samples;        /* nx ny nch nsamp of the request (nominal: rays that miss the grid
                                    have no samples and do no work) */
} rt_ticket_info;

rt_status rt_server_create(const rt_server_cfg *cfg, rt_server **out);
rt_status rt_submit(rt_server *sv, const rt_request *rq, uint64_t *ticket);
rt_status rt_poll(rt_server *sv, uint64_t ticket, rt_ticket_info *info);
rt_status rt_wait(rt_server *sv, uint64_t ticket, rt_ticket_info *info, uint64_t timeout_ns);
rt_status rt_cancel(rt_server *sv, uint64_t ticket);
/* Forget a finished ticket (done, failed or canceled): the server drops the
 * request's copies of its problem, and later rt_poll / rt_wait / rt_release
 * of that ticket return RT_ENOTFOUND.  A queued or running ticket gives
 * RT_EINVAL.  Without it a server keeps every ticket until rt_server_destroy. */
rt_status rt_release(rt_server *sv, uint64_t ticket);
rt_status rt_server_destroy(rt_server *sv);   /* drains admitted work, cancels the rest */

/* ---------------------------------------------------------------- 3-D spherical grid
 *
 * Non-axisymmetric fields (a hydrodynamic snapshot of T, n and v on a
 * spherical grid, as in the paper's runtime benchmark, Results "Runtime"):
 * the same LTE line physics and formal solution as the axisymmetric
 * renderer, with
 *   - nodes r_i = r_min (r_max/r_min)^(i/(nr-1)), theta_j = th_min + j (th_max -
 *     th_min)/(nt-1) (polar angle from +z), phi_k = 2 pi k / np (from +x
 *     towards +y); every field trilinear in (ln r, theta, phi) index space,
 *     clamped to the edge in r and theta, periodic in phi; n_H2 fades
 *     linearly to zero one cell beyond the radial and polar node ranges;
 *   - n_CO = x_CO n_H2 with x_CO a field (no surfaces, no mask);
 *   - v_los = v_sys + v . w, w = (0, sin i, -cos i), with v = v_r e_r +
 *     v_theta e_theta + v_phi e_phi (the polar and azimuthal terms vanish on
 *     the z axis);
 *   - each ray's chord through the sphere r <= r_max e^dln is cut into nsamp
 *     equal segments; camera, pixels and channels as in the axisymmetric
 *     renderer; inclination 0..180 deg (180: seen from -z).
 */
typedef struct {
    int32_t nr, nt, np;        /* nr, nt >= 2; np >= 1; nr nt np <= 2^28 */
    double r_min_au, r_max_au; /* 0 < r_min_au < r_max_au */
    double th_min, th_max;     /* polar angle of the first and last theta node [rad], 0 <= th_min < th_max <= pi */
} rt_grid3d;

/* Fields of the march: nodes = [nr][nt][np] records of 8 floats {ln n_H2
 * [cm^-3], T [K] (> 0), x_CO, v_r, v_theta, v_phi [km/s], 0, 0} as written by
 * rt_pack_fields3d (device, 16-byte aligned, nr nt np 32 bytes). */
typedef struct {
    rt_grid3d grid;
    const float *nodes;
    double v_turb;             /* turbulent Mach number, >= 0 */
    rt_line line;
    rt_camera cam;
    rt_spectral spec;
    int32_t nsamp;             /* samples per ray, >= 1 */
    double intensity_scale;    /* output = scale * I_nu */
} rt_problem3d;

/* Interleave six field planes [nr][nt][np] (device float32; ln_nh2, temp_k,
 * x_co required; NULL velocity planes are zero) into the node records of
 * rt_problem3d.nodes (device, caller-allocated nr nt np 8 floats, 16-byte
 * aligned).  RT_EINVAL on a bad grid or pointer. */
rt_status rt_pack_fields3d(const rt_grid3d *grid, const float *ln_nh2, const float *temp_k, const float *x_co,
                           const float *v_r, const float *v_theta, const float *v_phi, float *nodes, void *stream);

/* Render the cube [nch][ny][nx] (device float32) of a 3-D problem (Methods,
 * "Line Radiative Transfer": the discrete formal solution along each ray).
 * RT_OPT_CHANNEL_BLOCK and RT_OPT_RAY_SPLIT apply as in rt_render_cube;
 * 1 - e^-dtau is evaluated directly.  RT_EINVAL on invalid arguments,
 * RT_EDEVICE if a launch fails. */
rt_status rt_render_cube_3d(const rt_problem3d *p, float *cube, void *stream);
/* Work accounting of rt_render_cube_3d, as rt_render_census: counts[0] =
 * rays that cross the bounding sphere, counts[1] = their pixel-samples,
 * counts[2] = those thin in the march's sense, counts[3] = those with any
 * opacity, counts[4] = those inside the grid's fade (the march shades only
 * these in full); counts[2..4] are -1 when p->nodes is NULL or misaligned.
 * counts: [host] int64[5].  mask (device, [ny][nx] bytes, may be NULL).
 * Synchronous. */
rt_status rt_render_census_3d(const rt_problem3d *p, uint8_t *mask, int64_t *counts, void *stream);

/* ---------------------------------------------------------------- beam convolution
 *
 * A model cube is compared with an interferometric image at the image's
 * resolution (Methods, MCMC inference: model cubes against the observed
 * channel maps; the paper does not give the convolution, read here as
 * follows).  Every channel map is convolved with an elliptical Gaussian of
 * full widths at half maximum bmaj_px >= bmin_px (pixels), major axis at
 * position angle bpa_deg from +y towards -x, sampled at integer pixel offsets
 * within |dx|, |dy| <= R = ceil(3 bmaj_px / (2 sqrt(2 ln 2))), normalised to
 * unit sum; pixels outside the image count as zero.  The operator is its own
 * adjoint (point-symmetric kernel, zero padding): dL/din = rt_beam_convolve
 * of dL/dout.
 */
/* out = beam * in for a cube [nch][ny][nx] (device float32, nch <= 65535);
 * in and out must not overlap.  The weights live in a library-owned
 * per-stream scratch buffer.  RT_EINVAL on invalid sizes, beams or overlap,
 * RT_ENOMEM / RT_EDEVICE if the scratch or a launch fails. */
rt_status rt_beam_convolve(const float *in, float *out, int32_t nch, int32_t ny, int32_t nx, const rt_beam *beam,
                           void *stream);

/* ---------------------------------------------------------------- misc */
const char *rt_last_error(void);
int32_t rt_abi_version(void);

/* The cgs constants the library uses, in the order h, k_B, c, amu, au, pi
 * ([host] out[n]); returns how many exist. */
int32_t rt_constants(double *out, int32_t n);

/* Tuning knobs (process-wide).  RT_OPT_CHANNEL_BLOCK: channels per lane of
 * the forward march (8, 16, 24, 32, 48 or 64; 0 = automatic).
 * RT_OPT_THIN_EXPM1: 1 (default) evaluates 1 - e^-dtau of rt_render_cube's
 * march from its series on samples whose line-centre depth is small (below
 * 1/32 in natural units; every other kernel always does), 0 uses
 * 1 - e^-dtau directly everywhere (less accurate for optically thin lines,
 * kept for comparison).
 * RT_OPT_CKPT_SEGMENT: 0 (default) runs the adjoint's reverse march without
 * checkpoints, rebuilding each transmission from the ray's total optical
 * depth and the depth behind the sample; 2, 4, 8 or 16 selects the march
 * that stores the transmission every that many samples and recomputes each
 * segment from its checkpoint.  RT_OPT_ADJ_CHANNEL_BLOCK: channels per lane of
 * the adjoint's reverse march (8, 16, 24, 25 or 32; 0 = automatic; 24 and 25
 * only without checkpoints, 25 only with two lanes per pixel).  RT_OPT_ADJ_PIXEL_LANES: lanes sharing one pixel in the
 * checkpoint-free reverse march, each with its own channel block, their
 * per-sample sums added across the lanes (1, 2 or 4; 0 = automatic, which
 * takes 4 lanes of 16 or 12 channels in place of a pair of 32 or 24 when
 * the channels are uniformly spaced in those groups; 2 keeps the pair).
 * RT_OPT_RAY_SPLIT: lanes sharing one ray in the forward
 * march, each taking a consecutive sub-chord (1, 2, 4 or 8; 0 = automatic).
 * RT_OPT_GRAD_ACCUM: 0 (default) accumulates the gradients of the adjoint
 * (per-workgroup partials in LDS, then atomics into one accumulator per node)
 * in float, 1 in double; the partials are float either way.  RT_OPT_ADJ_SCRATCH_CAP: bytes of adjoint
 * scratch (sample tape, transmission checkpoints, cotangents) per pass; an
 * image whose scratch exceeds it is differentiated in bands of whole pixel
 * rows, at least one row per band (0 = default, 8 GiB).  The library keeps
 * that scratch with the stream it ran on and reuses it on later calls.
 * RT_OPT_FWD_GROUP: lanes per pixel of the forward march of 64-channel
 * blocks (1, 2 or 4; 0 = automatic): with G > 1 the G lanes of a pixel hold
 * 64/G channels each and share each sample's shading.  Used when the launch
 * shape is one 64-channel lane per pixel and each block's channel
 * velocities are uniformly spaced in groups of 64/G (lane m's = lane 0's +
 * m times one constant); otherwise one lane per pixel. */
enum { RT_OPT_CHANNEL_BLOCK = 1, RT_OPT_THIN_EXPM1 = 2, RT_OPT_CKPT_SEGMENT = 3, RT_OPT_RAY_SPLIT = 4,
       RT_OPT_GRAD_ACCUM = 5, RT_OPT_ADJ_SCRATCH_CAP = 6, RT_OPT_ADJ_CHANNEL_BLOCK = 7,
       RT_OPT_ADJ_PIXEL_LANES = 8, RT_OPT_FWD_GROUP = 9 };
rt_status rt_set_option(int32_t key, int64_t value);
int64_t rt_get_option(int32_t key);

#ifdef __cplusplus
}
#endif
#endif /* RTCUBE_H */
