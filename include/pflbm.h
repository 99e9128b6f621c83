/*
 * pflbm.h -- C ABI of the MI355X phase-field lattice Boltzmann library
 * (libpflbm.so, HIP for gfx950).
 *
 * The library advances a coupled two-phase solver one fused time step per
 * kernel launch: a hydrodynamic distribution g (D2Q9 or D3Q19, MRT collision
 * with the force F = F_s + F_b + F_p + F_mu, pressure-normalised equilibrium)
 * and a phase-field distribution h (D2Q5 or D3Q7, conservative Allen-Cahn or
 * Cahn-Hilliard). The method is the Fakhari2017 model of Li, Zhang, Wu, Peng,
 * Wang, "Comparative study and critical assessment of phase-field lattice
 * Boltzmann models ...", arXiv 2511.11360, Sec. II.C.1 (Eqs.
 * fakhari_model_simplified, fakhari_tau_model, mu_linear, fakhari_eqs,
 * fakhari_forces_modified, fakhari_update_all), with the Cahn-Hilliard phase
 * field of Sec. II.D.1 (Eqs. liang2_geq, liang2_G, backward-Euler time
 * derivative of Sec. III.B) as the second model. Naming: g here is the paper's
 * hydrodynamic f_beta, h the paper's phase-field g_alpha, W the paper's
 * interface width xi, M its mobility M_phi. phi_H = 1, phi_L = 0.
 *
 * Conventions shared by every call
 *  - Every function returns an int status: PFLBM_OK (0) or a negative
 *    PFLBM_E* code. Nothing throws or aborts across the ABI. After an error on
 *    a handle, pflbm_last_error() returns a message owned by the handle.
 *    PFLBM_EINVAL and PFLBM_EUNSUPPORTED (a rejected call: nothing launched)
 *    leave the handle as it was. After PFLBM_EHIP every later
 *    call returns PFLBM_ESTATE until the handle is destroyed. After
 *    PFLBM_EUNSTABLE every later call returns PFLBM_ESTATE until
 *    pflbm_init() or pflbm_load_state() replaces the state (recovery from a
 *    checkpoint).
 *  - Field pointers are DEVICE pointers to float64 arrays in canonical
 *    layout, x fastest: scalars [z][y][x], vectors [d][z][y][x] with
 *    d = 2 (2-D) or 3, distributions [q][z][y][x] in the canonical population
 *    order below. The caller owns them; the library never keeps them.
 *  - The library allocates no device memory. Its whole device state (g, the
 *    two h buffers, the CH (phi u) state, reduction scratch) lives in one
 *    caller-owned device buffer of pflbm_state_bytes() bytes passed to
 *    pflbm_create(), which the caller must keep alive until pflbm_destroy().
 *  - Calls are asynchronous on the HIP stream given to pflbm_create(), except
 *    those documented as synchronising.
 *  - Node (i, j, k) sits at (x, y, z) = (i, j, k). A walled axis has its walls
 *    half a spacing outside its first and last node (halfway bounce-back).
 *
 * Canonical population order
 *  D2Q9 : 0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
 *         5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1)
 *  D2Q5 : the first five D2Q9 vectors; weights 1/3, 1/6
 *  D3Q19: 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z, 7 (+x+y), 8 (-x-y),
 *         9 (+x-y), 10 (-x+y), 11 (+x+z), 12 (-x-z), 13 (+x-z), 14 (-x+z),
 *         15 (+y+z), 16 (-y-z), 17 (+y-z), 18 (-y+z)
 *  D3Q27: the nineteen D3Q19 vectors, then the corners 19 (+x+y+z), 20 (-x-y-z),
 *         21 (+x+y-z), 22 (-x-y+z), 23 (+x-y+z), 24 (-x+y-z), 25 (-x+y+z),
 *         26 (+x-y-z); weights 8/27, 2/27, 1/54, 1/216
 *  D3Q7 : the first seven D3Q19 vectors; with c_s^2 = 1/3 (Sec. IV) the rest
 *         weight is 0 and the face weights 1/6, so for the AC model the rest
 *         population of h is identically zero and is not stored.
 */
#ifndef PFLBM_H
#define PFLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PFLBM_OK            0
#define PFLBM_EINVAL       -1   /* invalid argument; handle state unchanged */
#define PFLBM_EUNSUPPORTED -2   /* valid but not supported by this library */
#define PFLBM_EHIP         -3   /* HIP runtime error (sticky) */
#define PFLBM_EUNSTABLE    -4   /* NaN/Inf in phi or u, or rho <= 0, detected */
#define PFLBM_ESTATE       -5   /* handle in an error state */

/* lattice pair: hydrodynamic g + phase-field h */
#define PFLBM_D2Q9_D2Q5   0
#define PFLBM_D3Q19_D3Q7  1
#define PFLBM_D3Q27_D3Q7  2   /* the paper's 3-D hydrodynamic lattice (Sec. IV) */

/* phase-field model */
#define PFLBM_AC 0   /* conservative Allen-Cahn, Eqs. fakhari_geq, fakhari_G_modified */
#define PFLBM_CH 1   /* Cahn-Hilliard, Eqs. liang2_geq, liang2_G */
#define PFLBM_L18 3  /* Liang2018 (Sec. II.C): conservative AC with Eqs. liang_geq and
                        liang_G_final (backward-Euler d(phi u)/dt) and its conservative-form
                        hydrodynamics, Eqs. liang_feq, liang_F_final, liang_velocity_update,
                        liang_p_update. Stationary walls only; with fp16-stored g,
                        rho_H and rho_L <= 16 (f / w must fit the fp16 range) */
#define PFLBM_L14 4  /* Liang2014 with its hydrodynamics (Sec. II.D.1): the CH phase field of
                        PFLBM_CH with Eqs. liang2_feq, liang2_F (Gamma, s of Eq. Gamma_beta),
                        F_a = (rho_H - rho_L) M lap(mu_phi) u, the velocity update of
                        Eq. liang2014_velocity_update and the pressure of Eq. liang_p_update;
                        the step kernel forms mu_phi itself around each tile for its
                        Laplacian. Same wall and fp16 limits as PFLBM_L18 */
#define PFLBM_NL 2   /* nonlocal Allen-Cahn, Eqs. Chai_geq, chai_G (Chai2018), the source
                        blended with the conservative flux by lam as in Eq. Hu_G (Hu2019);
                        phi = sum h + (1 - lam) R / 2 (Eq. chai2018_phi_update), with the
                        multiplier gamma of Eq. lagrange_multiplier reduced over the whole
                        box in float64 before every step */

/* storage / arithmetic form */
#define PFLBM_FP64        0  /* g, h float64; float64 arithmetic */
#define PFLBM_FP32        1  /* g, h float32; float32 arithmetic */
#define PFLBM_MIXED_FP16  2  /* g stored as fp16 of 4096 g_i / w_i, h float32; float32 arithmetic */
#define PFLBM_MIXED_BF16  3  /* g stored as bf16 of g_i / w_i, h float32; float32 arithmetic */
/* In both 16-bit forms the step rounds the stored g stochastically (unbiased:
   up or down with probabilities that make the expectation the float32 value),
   from random bits keyed by node, step and population, so runs are
   reproducible and independent of the tile and z block; initialisation and
   pflbm_set_distributions round to nearest even, and so does every store of
   PFLBM_L14 (its kernel has no registers to spare for the random words). */

/* step-kernel tile: x nodes by y rows per workgroup, one node per thread
   (3-D; the 2-D lattice always uses 64 x 4). Results do not depend on it. */
#define PFLBM_TILE_AUTO   0  /* 256x4 for float32 and the fp16/bf16-stored forms
                                at nx >= 256 (PFLBM_L14 with 16-bit g: 128x8 on
                                D3Q19, 64x4 on D3Q27), 128x2 for float64;
                                narrower when nx is */
#define PFLBM_TILE_64x4   1  /* 256 threads; workgroups ordered so each XCD
                                sweeps a contiguous run */
#define PFLBM_TILE_128x2  2  /* 256 threads, hardware workgroup order */
#define PFLBM_TILE_256x1  3  /* 256 threads, hardware workgroup order */
#define PFLBM_TILE_256x4  4  /* 1024 threads, ordered as 64x4 */
#define PFLBM_TILE_128x8  5  /* 1024 threads, ordered as 64x4 */

/* boundary per axis */
#define PFLBM_PERIODIC 0
#define PFLBM_WALL     1    /* halfway bounce-back; at most one walled axis */

/* viscosity interpolation */
#define PFLBM_VISC_LINEAR_MU 0   /* Eq. mu_linear: mu linear in phi, nu = mu / rho */
#define PFLBM_VISC_LINEAR_NU 1   /* Eq. fakhari_mu_update: nu linear in phi */

typedef struct pflbm_params {
    int lattice;          /* PFLBM_D2Q9_D2Q5, PFLBM_D3Q19_D3Q7 or PFLBM_D3Q27_D3Q7 */
    int model;            /* PFLBM_AC, PFLBM_CH, PFLBM_NL, PFLBM_L18 or PFLBM_L14 */
    int precision;        /* PFLBM_FP64 ... PFLBM_MIXED_BF16 */
    int nx, ny, nz;       /* nodes per axis, each >= 1; nz == 1 for 2-D */
    int bc[3];            /* PFLBM_PERIODIC or PFLBM_WALL per axis x, y, z */
    double wall_u[2][3];  /* velocity of the low / high wall of the walled axis;
                             must be tangential to the wall */
    double rho_H, rho_L;  /* phase densities, > 0 (Eq. fakhari_rho_update) */
    double nu_H, nu_L;    /* kinematic viscosities; tau = 3 nu + 1/2 > 1/2
                             (Eq. fakhari_tau_model) */
    int visc_interp;      /* PFLBM_VISC_LINEAR_MU (paper's default) or _NU */
    double M;             /* mobility, > 0; tau_phi = 3 M + 1/2 (AC),
                             3 M / eta + 1/2 (CH) */
    double W;             /* interface width xi, > 0 */
    double sigma;         /* surface tension, >= 0; beta = 12 sigma / W,
                             kappa = 3 sigma W / 2 (Eqs. coefficient1, coefficients) */
    double eta;           /* CH mobility parameter of Eq. liang2_geq, > 0 */
    double gravity[3];    /* body acceleration: F_b = rho * gravity */
    double force[3];      /* uniform force density added to F_b (Sec. III.D drive) */
    double s_other;       /* MRT rate of every non-stress moment, in (0, 2) */
    double normal_eps;    /* interface normal n = grad phi / sqrt(|grad phi|^2 + eps^2), >= 0;
                             0 is the paper's n = grad phi / |grad phi| of
                             Eq. fakhari_G_modified with n = 0 where grad phi = 0 */
    double lam;           /* PFLBM_NL: weight of the conservative flux in [0, 1]
                             (0 = Chai2018, Hu2019 uses 0.9); ignored otherwise */
    int freeze_phi;       /* nonzero: h (hence phi) is not updated (Sec. III.D) */
    int check_interval;   /* every this many steps pflbm_step checks for NaN/Inf
                             or rho <= 0 (synchronising); 0 = never */
    int zblock;           /* z planes per workgroup, 0 = automatic: the step kernel
                             then sizes its grid from the device occupancy
                             (tuning only) */
    int tile;             /* step-kernel tile, PFLBM_TILE_* (tuning only: results
                             do not depend on it) */
} pflbm_params;

/* FP64 diagnostics of one state (Eq. volume_continuous; volume by counting
   phi > 1/2 of Sec. IV.A; delta phi_max of Sec. III.A from phi_min/phi_max;
   umax = max |u|; mean pressure inside r < R - 2W and outside r > R + 2W). */
typedef struct pflbm_diag {
    double V_phi;      /* sum (phi - phi_L) / (phi_H - phi_L) */
    double V_count;    /* number of nodes with phi > 1/2 */
    double sum_phi;
    double phi_min, phi_max;
    double umax;
    double p_in, p_out;        /* NaN when the region is empty or no centre given */
    long long n_in, n_out;
    int unstable;              /* 1 if NaN/Inf in phi or u, or rho <= 0, anywhere */
} pflbm_diag;

typedef struct pflbm pflbm_t;

/* Bytes of the device state buffer for these parameters. Host pointers.
   The buffer holds two copies of each distribution in its storage form
   (plane-major [z][q][y][x], planes padded to a multiple of 64 nodes): a step
   reads the previous step's post-collision populations from one, pulling
   population i of node x from node x - c_i, and writes its own post-collision
   populations at x into the other. */
int pflbm_state_bytes(const pflbm_params* params, size_t* bytes);

/* Validate params and bind a handle to the caller's device buffer dev_state
   (bytes >= pflbm_state_bytes, 256-byte aligned) and HIP stream hip_stream
   (hipStream_t, NULL = default stream) on the current device. *out receives a
   host-allocated handle, freed by pflbm_destroy(). */
int pflbm_create(const pflbm_params* params, void* hip_stream, void* dev_state,
                 size_t bytes, pflbm_t** out);

/* Equilibrium initialisation: h = h_eq(phi0, u0) (CH with mu_phi(phi0)),
   g = g_eq(p0 / (rho0 c_s^2), u0); resets the step counter. phi0 [z][y][x],
   u0 [d][z][y][x] or NULL (zero), p0 [z][y][x] or NULL (zero): device float64. */
int pflbm_init(pflbm_t* h, const double* phi0, const double* u0, const double* p0);

/* Advance nsteps >= 0 fused time steps (one kernel launch each). Returns
   PFLBM_EUNSTABLE (and stops, with the failing state current) when a check
   due under check_interval finds NaN/Inf in phi or u, or rho <= 0. */
int pflbm_step(pflbm_t* h, int nsteps);

/* One step, as pflbm_step(h, 1), that also writes the state it starts from:
   g and hd as pflbm_get_distributions would have returned them just before
   the step, and pu (if not NULL) as pflbm_get_phiu would have (CH, Liang2018,
   Liang2014; ignored for the other models). Device pointers, canonical
   layouts; the _f32 form writes float32 g, hd and pu (the forward state of
   the float32 adjoint). The read-out rides on the step's own pull of the state,
   so the backward pass of a checkpointed run needs no separate read-out.
   Float64 and float32 storage forms only (PFLBM_EUNSUPPORTED otherwise). */
int pflbm_step_record(pflbm_t* h, double* g, double* hd, double* pu);
int pflbm_step_record_f32(pflbm_t* h, float* g, float* hd, float* pu);

/* Macroscopic fields of the current state (the values the next step uses):
   phi, u (d components), p = rho c_s^2 sum g, rho. Device float64 outputs,
   any may be NULL. */
int pflbm_fields(pflbm_t* h, double* phi, double* u, double* p, double* rho);

/* Diagnostics of the current state, reduced in float64 on the device with a
   fixed order (bit-reproducible). centre: HOST array of dim doubles or NULL;
   R: droplet radius for the pressure regions. Synchronises the stream. */
int pflbm_volume(pflbm_t* h, const double* centre, double R, pflbm_diag* out);

/* Copy the post-streaming distributions out as canonical float64 (decoding
   the storage form and applying the pending streaming). Device pointers
   g [Qg][z][y][x] and hd [Qh][z][y][x] (Qh = 5 or 7, rest included). */
int pflbm_get_distributions(pflbm_t* h, double* g, double* hd);

/* The same read-out in float32 (g and hd float32 arrays of the same layout),
   the forward state of the float32 adjoint. */
int pflbm_get_distributions_f32(pflbm_t* h, float* g, float* hd);

/* Overwrite the state from canonical float64 distributions (device pointers,
   same layout as pflbm_get_distributions); the storage form rounds them.
   For AC on D3Q7 the rest population of h must be zero. CH keeps its (phi u)
   state. */
int pflbm_set_distributions(pflbm_t* h, const double* g, const double* hd);

/* The (phi u) of the previous step that the CH, Liang2018 and Liang2014
   models keep for their backward-Euler d(phi u)/dt (Eq. liang2_G): copied
   out to, or overwritten from, canonical float64 pu [3][z][y][x] (device
   pointer; the third component of a 2-D box is zero). Set rounds to the
   compute type (float32 for the reduced forms). PFLBM_EUNSUPPORTED for the
   AC and nonlocal models. Asynchronous. */
int pflbm_get_phiu(pflbm_t* h, double* pu);
int pflbm_set_phiu(pflbm_t* h, const double* pu);

/* Number of completed steps since pflbm_init. */
int pflbm_step_count(const pflbm_t* h, long long* steps);

/* Checkpoint: raw copy of the native state (distributions in their storage
   form, step counter, CH state) to/from a caller-owned device
   buffer of pflbm_checkpoint_bytes() bytes. Its 256-byte header records the
   checkpoint size and the layout it was written with (lattice, model,
   precision, frozen phase field, nx, ny, nz); pflbm_load_state reads the
   header first (synchronising the stream) and returns PFLBM_EINVAL, copying
   nothing, when any of them differs from the handle's. The physical
   parameters (sigma, M, W, ...) may differ. */
int pflbm_checkpoint_bytes(const pflbm_t* h, size_t* bytes);
int pflbm_save_state(pflbm_t* h, void* dev_dst);
int pflbm_load_state(pflbm_t* h, const void* dev_src);

/* Discrete adjoint (every model). The adjoint of one time step X^n -> X^{n+1}
   (X = canonical float64 post-streaming distributions, as returned by
   pflbm_get_distributions) given lambda^{n+1} = dL/dX^{n+1}: writes
   lambda^n = dL/dX^n and ADDS dL/d(sigma, M, W) of this step into dparams
   (device float64[3], may be NULL). fwd_g/fwd_h hold X^n. All pointers are
   device pointers in canonical layout ([Qg][z][y][x], [Qh][z][y][x]);
   lam_*_out must not alias lam_*. work: caller-owned device workspace of
   pflbm_adjoint_workspace_bytes(). Uses the handle's parameters; float64
   arithmetic whatever the handle's precision. The method's reverse mode is
   not in the paper: it is the exact transpose of the discrete step of
   Sec. II.C.1 (AC), Sec. II.D.1 (CH), Secs. II.C.3-4 (nonlocal AC, Eqs.
   nonlocalAC, lagrange_multiplier, Chai_geq, Hu_G, with its global
   multiplier), Sec. II.C.2 (Liang2018, Eqs. liang_feq, liang_F_final,
   liang_velocity_update, liang_p_update, liang_geq, liang_G_final) or Sec.
   II.D.1 with its hydrodynamics (Liang2014, Eqs. liang2_feq, liang2_F,
   liang2014_velocity_update, whose F_a reads lap mu_phi) as implemented
   here, on every lattice pair. The CH, Liang2018 and Liang2014 states also
   hold (phi u) of the previous step, so those models go through
   pflbm_adjoint_step_pu; pflbm_adjoint_step returns PFLBM_EUNSUPPORTED for
   them, and both return PFLBM_EUNSUPPORTED for a frozen phase field. The
   nonlocal model's workspace holds two more per-node arrays, Liang2014's
   four more. */
int pflbm_adjoint_workspace_bytes(const pflbm_t* h, size_t* bytes);
int pflbm_adjoint_step(pflbm_t* h, const double* fwd_g, const double* fwd_h,
                       const double* lam_g, const double* lam_h,
                       double* lam_g_out, double* lam_h_out, double* dparams, void* work);

/* The adjoint step with the (phi u) part of the state X = (g, h, pu) of the
   CH and Liang2014 models (Eqs. liang2_geq, liang2_G with the backward-Euler
   d(phi u)/dt) and of the Liang2018 model (Eq. liang_G_final):
   fwd_pu holds (phi u) of the step before X^n (pflbm_get_phiu), lam_pu its
   adjoint dL/dpu^{n+1}, lam_pu_out receives dL/dpu^n; all [3][z][y][x]
   device float64, lam_pu_out not aliasing lam_pu. For the AC and nonlocal
   models the three pu pointers are ignored (may be NULL) and the call equals
   pflbm_adjoint_step. */
int pflbm_adjoint_step_pu(pflbm_t* h, const double* fwd_g, const double* fwd_h, const double* fwd_pu,
                          const double* lam_g, const double* lam_h, const double* lam_pu,
                          double* lam_g_out, double* lam_h_out, double* lam_pu_out,
                          double* dparams, void* work);

/* The float32 adjoint of the AC step (Sec. II.C.1) and, through the _pu
   forms, of the CH step (Sec. II.D.1): the passes of pflbm_adjoint_step and
   pflbm_adjoint_step_pu in float32 arithmetic on float32 arrays of the same
   layouts (the forward state as pflbm_get_distributions_f32 or
   pflbm_step_record_f32 gives it); the parameter terms are still reduced,
   and ADDED into dparams, in float64.
   The phase field of the forward state, its stencils, phi (1 - phi), the
   cubic term of mu and the non-equilibrium h_eq - h are formed in float64
   (float32 differences of them cancel inside a droplet); everything else
   carries float32 rounding. It moves 368 bytes per node against the float64
   adjoint's 720 (CH: 404 against 792). work: the workspace of pflbm_adjoint_workspace_bytes().
   pflbm_adjoint_seed_phi_f32 and pflbm_adjoint_init_f32 are the float32 forms
   of the seed and of the initialisation adjoint (phi0, u0, p0 float64, as
   for pflbm_init); pflbm_adjoint_step_pu_f32 and pflbm_adjoint_init_pu_f32
   are those of the CH model, with the (phi u) arrays of pflbm_adjoint_step_pu
   in float32. PFLBM_EUNSUPPORTED for the other models, and for a form that
   does not match the model (the AC model has no (phi u), the CH model needs
   it). */
int pflbm_adjoint_step_f32(pflbm_t* h, const float* fwd_g, const float* fwd_h,
                           const float* lam_g, const float* lam_h,
                           float* lam_g_out, float* lam_h_out, double* dparams, void* work);
int pflbm_adjoint_seed_phi_f32(pflbm_t* h, const float* dphi, float* lam_g, float* lam_h);
int pflbm_adjoint_init_f32(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                           const float* lam_g, const float* lam_h, float* dphi0);
int pflbm_adjoint_step_pu_f32(pflbm_t* h, const float* fwd_g, const float* fwd_h, const float* fwd_pu,
                              const float* lam_g, const float* lam_h, const float* lam_pu, float* lam_g_out,
                              float* lam_h_out, float* lam_pu_out, double* dparams, void* work);
int pflbm_adjoint_init_pu_f32(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                              const float* lam_g, const float* lam_h, const float* lam_pu, float* dphi0,
                              double* dparams, void* work);

/* The same adjoint step for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   allocation): no workspace argument; the step uses a scratch array that the
   library holds on each device it runs on, PFLBM_ADJOINT_SCRATCH_BYTES bytes
   (enough for boxes of up to 128^3 = 2097152 nodes), until the process ends.
   Returns PFLBM_EINVAL, launching nothing, when pflbm_adjoint_workspace_bytes
   exceeds that. It allocates nothing. Calls that overlap on one device (on
   different streams, or from different handles) share the array and race;
   calls in order on one stream are safe. Results equal pflbm_adjoint_step's
   bit for bit. AC model (PFLBM_EUNSUPPORTED otherwise). */
#define PFLBM_ADJOINT_SCRATCH_BYTES 100925440
int pflbm_adjoint_step_noalloc(pflbm_t* h, const double* fwd_g, const double* fwd_h,
                               const double* lam_g, const double* lam_h,
                               double* lam_g_out, double* lam_h_out, double* dparams);

/* Seed of the adjoint from a loss on the phase field of a state: given
   dL/dphi [z][y][x] (device float64), writes lambda = dL/dX for that state,
   lam_g [Qg][z][y][x] = 0 and lam_h [Qh][z][y][x] = dL/dphi for every
   population, the transpose of phi = sum_a h_a (Eq. fakhari_phi_update).
   Every model but the nonlocal one (PFLBM_EUNSUPPORTED there: its phase
   field is corrected, use pflbm_adjoint_seed); for the models with a (phi u)
   state the loss does not depend on pu, so lam_pu of that state is zero (the
   caller's buffer). Asynchronous. */
int pflbm_adjoint_seed_phi(pflbm_t* h, const double* dphi, double* lam_g, double* lam_h);

/* The seed for every model with an adjoint: dphi = dL/dphi of the phase field
   that pflbm_fields returns for the state whose canonical h is fwd_h. For the
   nonlocal model that field is phi* = sum h + (1 - lam) R / 2 (the corrected
   phi of Sec. II.C.3), which depends on every node through the multiplier
   gamma of Eq. lagrange_multiplier and on M and W through the source R: the
   seed applies its transpose and ADDS the M and W terms into dparams (device
   float64[3], may be NULL); work: workspace of
   pflbm_adjoint_workspace_bytes(). For the other models it equals
   pflbm_adjoint_seed_phi (fwd_h, dparams and work unused). */
int pflbm_adjoint_seed(pflbm_t* h, const double* fwd_h, const double* dphi, double* lam_g, double* lam_h,
                       double* dparams, void* work);

/* dL/dphi0 of the equilibrium initialisation (pflbm_init) given
   lambda^0 = dL/dX^0: dphi0 [z][y][x] (device float64, overwritten). u0 and
   p0 as passed to pflbm_init (NULL = zero). AC and nonlocal models (the
   models with a (phi u) state go through pflbm_adjoint_init_pu). */
int pflbm_adjoint_init(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                       const double* lam_g, const double* lam_h, double* dphi0);

/* The same with the (phi u) part: lam_pu = dL/dpu^0 [3][z][y][x]. The CH
   (and Liang2014) initialisation h = h_eq(phi0, mu_phi(phi0), u0) (Eq.
   liang2_geq, mu_phi of Eq. chemical_potential, on the step's Laplacian
   stencil), pu^0 = phi0 u0 (Liang2014: f = f_eq of Eq. liang2_feq at
   rho(phi0)), depends on sigma and W through mu_phi: their terms are ADDED
   into dparams (device float64[3], may be NULL). work: workspace of
   pflbm_adjoint_workspace_bytes(). Liang2018: f = f_eq of Eq. liang_feq at
   rho(phi0), h of Eq. liang_geq, pu^0 = phi0 u0 (no parameter terms; dparams
   and work unused). For the AC and nonlocal models lam_pu, dparams and work
   are ignored and the call equals pflbm_adjoint_init. */
int pflbm_adjoint_init_pu(pflbm_t* h, const double* phi0, const double* u0, const double* p0,
                          const double* lam_g, const double* lam_h, const double* lam_pu,
                          double* dphi0, double* dparams, void* work);

/* Measurement only (no part of the method): memory-pattern probes of the
   mixed-precision D3Q19 + D3Q7 step's HBM streams, 19 fp16 g and 6 fp32 h
   populations per node read once and written once in the step's plane-major
   layout [z][q][plane] (plane = nx ny rounded up to 64 nodes), with no
   arithmetic. They give the bandwidth ceiling of the step kernel's access
   pattern on the device at hand. g_src / g_dst hold g_bytes, h_src / h_dst
   h_bytes of device memory (pflbm_probe_bytes); one launch per call on
   hip_stream (hipStream_t), asynchronous; zblock = z planes per workgroup
   (the step kernel's automatic depth reproduces its grid). Returns
   PFLBM_EINVAL for bad sizes or pattern, PFLBM_EHIP if the launch fails. */
#define PFLBM_PROBE_CHUNKS    0  /* contiguous 1024-node chunks of every population plane */
#define PFLBM_PROBE_TILES     1  /* 256 x 4 tiles in XCD runs, z blocks marched, aligned */
#define PFLBM_PROBE_SHIFT_LD  2  /* PFLBM_PROBE_TILES, g populations with c_x != 0 loaded
                                    from x - c_x (the pull streaming of the step) */
#define PFLBM_PROBE_SHIFT_ST  3  /* PFLBM_PROBE_TILES, those populations stored at x + c_x
                                    (the shifted stores of in-place streaming) */
#define PFLBM_PROBE_ZSKEW     4  /* PFLBM_PROBE_SHIFT_LD; when one z block spans the box,
                                    each workgroup starts at its own plane and wraps */
int pflbm_probe_bytes(int nx, int ny, int nz, size_t* g_bytes, size_t* h_bytes);
int pflbm_probe_stream(const void* g_src, void* g_dst, const void* h_src, void* h_dst, int nx,
                       int ny, int nz, int pattern, int zblock, void* hip_stream);

void pflbm_destroy(pflbm_t* h);
const char* pflbm_last_error(const pflbm_t* h);
const char* pflbm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* PFLBM_H */
