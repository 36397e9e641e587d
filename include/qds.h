/*
 * libqds — quasi-cylindrical direction-splitting (QDS) field advance with the
 * Klein-Gordon axion solver and the axion-regenerated fields, for MI355X (gfx950).
 *
 * Method: "X-dispersionless solver for electromagnetic and axion fields in a
 * cylindrical particle-in-cell code" (arXiv 2609.03550).  Every retained
 * azimuthal mode m of the fields (Eq. fourier_decomp) lives on a staggered
 * (x, r) grid; the transverse transport variables T_r^+- = E_r +- B_theta,
 * T_theta^+- = E_theta +- B_r (Eq. Tdefs) move exactly one cell per step
 * (c dt = dx, Eqs. Trp_update..Ttm_update), E_x and B_x leapfrog (Eq.
 * Ex_update), the axion transport variables T_a^+- and phi follow Eqs.
 * Ta_plus_update, Ta_minus_update, phi_update, and a duplicate set of fields
 * is driven by the axion current j_a (Eqs. jax_mode, jar_mode, jat_mode).
 *
 * Units: c = eps0 = mu0 = 1.  The axion and regenerated fields are carried
 * scaled (phi/g, E1/g^2) when s_phi = s_j = 1, so the coupling never appears.
 *
 * Conventions for every entry point:
 *  - Device pointers are HIP device memory owned by the caller unless stated.
 *  - Work is enqueued on ``stream`` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous; argument errors are returned synchronously before
 *    anything is enqueued.  A launch failure is returned as QDS_EHIP.
 *  - A handle must not be used from two host threads at once, and its calls
 *    must be ordered on the device: issue them on one stream, or synchronise
 *    before switching streams (the handle keeps a device-side argument table
 *    that a call may refresh).
 *  - On any error, qds_last_error(handle) holds a message (never NULL).
 */
#ifndef QDS_H
#define QDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QDS_OK = 0,
    QDS_EINVAL = 1,        /* bad argument (sizes, flags, null pointers) */
    QDS_ECFL = 2,          /* c dt != dx, or the radial stability bound fails */
    QDS_ENOMEM = 3,        /* library-owned allocation failed */
    QDS_EHIP = 4,          /* a HIP call or kernel launch failed */
    QDS_EUNSUPPORTED = 5,  /* combination not built (e.g. more than 8 modes) */
    QDS_ESTATE = 6         /* state descriptor inconsistent with the handle */
} qds_status;

enum { QDS_F64 = 0, QDS_F32 = 1 };
enum { QDS_X_OPEN = 0, QDS_X_PERIODIC = 1, QDS_X_WINDOW = 2 };
enum { QDS_R_OPEN = 0, QDS_R_PEC = 1 };
enum { QDS_HAS_PLASMA = 1, QDS_HAS_AXION = 2, QDS_HAS_AREM = 4 };
enum { QDS_J_NONE = 0, QDS_J_RING = 1, QDS_J_PARTICLES = 2 };

/* Planes of the state (each [modes][nr+1][ld] complex, x contiguous). */
enum {
    QDS_P_TRP = 0,   /* T_r^+ at (x_i, r_{j+1/2}, t^n); row nr holds the exterior ghost B_theta(r_{nr+1/2}) */
    QDS_P_TRM = 1,   /* T_r^- at (x_i, r_{j+1/2}, t^n); row nr unused */
    QDS_P_TTP = 2,   /* T_theta^+ at (x_i, r_j, t^n), rows 0..nr */
    QDS_P_TTM = 3,   /* T_theta^- at (x_i, r_j, t^n) */
    QDS_P_EX = 4,    /* E_x at (x_{i+1/2}, r_j, t^{n-1/2}) */
    QDS_P_BX = 5,    /* B_x at (x_{i+1/2}, r_{j+1/2}, t^{n-1/2}); row nr = exterior ghost */
    QDS_P_JX = 6,    /* plasma j_x at (x_{i+1/2}, r_j, t^{n-1}) */
    QDS_P_JR = 7,    /* plasma j_r at (x_i, r_{j+1/2}, t^{n-1/2}) */
    QDS_P_JT = 8,    /* plasma j_theta at (x_i, r_j, t^{n-1/2}) */
    /* 9..17: the same nine planes for the regenerated set (QDS_P_SET1 + k) */
    QDS_P_SET1 = 9,
    QDS_P_PHI = 18,  /* phi at (x_{i+1/2}, r_{j+1/2}, t^n); row nr = exterior ghost phi */
    QDS_P_TAP = 19,  /* T_a^+ at (x_i, r_{j+1/2}, t^{n-1/2}) */
    QDS_P_TAM = 20,  /* T_a^- at (x_i, r_{j+1/2}, t^{n-1/2}) */
    QDS_NPLANES = 21
};

/* Grid and field content.  x columns i = 0..nx-1 (x_i = i dx); half-x columns
 * hold x_{i+1/2}, the last one (i = nx-1) outside the domain and zero unless
 * x is periodic.  Radial rows r_j = j dr (j = 0..nr) and r_{j+1/2}. */
typedef struct {
    int32_t nx;        /* >= 8 */
    int32_t nr;        /* >= 4 */
    int32_t dtype;     /* QDS_F64 | QDS_F32 (complex interleaved re, im) */
    int32_t x_bc;      /* QDS_X_OPEN | QDS_X_PERIODIC | QDS_X_WINDOW (one cell per step) */
    int32_t r_bc;      /* QDS_R_OPEN (outflow, Sec. 3.2) | QDS_R_PEC (conducting wall, tests) */
    int32_t content;   /* QDS_HAS_* bits: which planes the state holds */
    double dr;
} qds_grid;

/* Current model: cold-plasma response d_t j = wp2 E on every set, plus an
 * optional prescribed j_x^(0) drive standing in for deposition:
 *   j_x = amp exp(-(x - x0 - v t)^2 / 2 sx^2) exp(-(r - r0)^2 / 2 sr^2) (1 + noise xi),
 * xi a SplitMix64 + Box-Muller normal per (step, lab column, row) from seed. */
typedef struct {
    double wp2;
    int32_t kind;      /* QDS_J_NONE | QDS_J_RING | QDS_J_PARTICLES */
    int32_t pad_;
    double amp, x0, v, sx, r0, sr, noise;
    uint64_t seed;
    /* QDS_J_PARTICLES: currents deposited by qds_particles_step, added to the
     * background set (planes in the layout of a state plane, the handle's
     * dtype): j_x^n = (pjx_prev + pjx_next)/2 with pjx_prev the deposit of the
     * step ending at t^{n-1/2} (may be NULL: taken as zero) and pjx_next that
     * of the step ending at t^{n+1/2}; j_r and j_theta of the latter (pjr,
     * pjt, on integer columns) are averaged along x onto the source points
     * x_{i+1/2} (Sec. 3.1, last paragraph).  On the fused kernels the library
 * forms these sums once per call into three planes of its own (allocated on
 * first use), which the background march reads as its extra currents. */
    const void* pjx_prev;
    const void* pjx_next;
    const void* pjr;
    const void* pjt;
} qds_current;

/* Axion parameters (ignored unless the grid content has QDS_HAS_AXION). */
typedef struct {
    double ma2;        /* (m_a c^2 / hbar)^2 in code units */
    double s_phi;      /* scale of the KG source E.B (1 in scaled units) */
    double s_j;        /* scale of j_a (1 in scaled units) */
    double bext[6];    /* uniform external B added to the background in S_a and j_a:
                          re/im of B_x^(0), B_r^(1), B_theta^(1) */
} qds_axion;

/* State: two caller-owned device buffers of qds_state_bytes() bytes each.
 * ``cur`` names the one holding the current state; qds_step advances it,
 * the step counter and the moving-window offset. */
typedef struct {
    void* buf[2];
    int32_t cur;
    int32_t pad_;
    int64_t step;      /* n: the state is at t^n = n dt */
    int64_t window;    /* cells the moving window has advanced */
} qds_state;

typedef struct qds_ctx* qds_handle;

/* Largest eigenvalues of the discrete radial operators over modes 0..modes-1
 * (host only, no device work).  With c dt = dx the one-step map of the
 * scheme factorises per mode and axial wavenumber k (Sec. 2.1: exact x
 * transport, explicit radial sources) as
 *   sin^2(w dt/2) = sin^2(k dx/2) + (dt/2)^2 mu cos^2(k dx/2),
 * mu an eigenvalue of the radial operator of E_x (integer rows) or B_x
 * (half rows); the Klein-Gordon step (Sec. 2.2) likewise with mu + m_a^2 of
 * the operator of phi.  *mu_em is the electromagnetic maximum, *mu_kg the
 * Klein-Gordon one without m_a^2.  r_bc = QDS_R_PEC gives the exact values
 * for a conducting wall; QDS_R_OPEN the larger of the outer row with and
 * without its exterior flux.  QDS_EINVAL for nr < 2, dr <= 0, modes outside
 * 1..8 or a bad r_bc. */
qds_status qds_radial_mu_max(int32_t nr, double dr, int32_t modes, int32_t r_bc, double* mu_em, double* mu_kg);

/* Create a handle.  ``modes`` retained azimuthal modes m = 0..modes-1 (1..8).
 * Fails with QDS_ECFL unless |dt - dx| <= 4 ulp(dx) (exact one-cell shift,
 * Sec. 2.1) and dt^2 mu_em <= 4 (qds_radial_mu_max: the step is stable
 * exactly then).  qds_step fails with QDS_ECFL when the axion is advanced
 * and dt^2 (mu_kg + m_a^2) > 4.  Allocates
 * the library's own scratch in device memory: with the regenerated set, four
 * planes (the three axion-current components and the axion source S_a).
 * Later allocations of the handle, on first use: the pair buffer
 * (qds_state_bytes plus three planes, QDS_OPT_PAIR with the regenerated set),
 * two mode-0 drive planes (a prescribed drive on the fused kernels), three
 * particle-current planes (QDS_J_PARTICLES on the fused kernels). */
qds_status qds_init(const qds_grid* grid, int32_t modes, double dx, double dt, qds_handle* out);

/* Bytes of one state buffer, the row pitch in elements, and the byte offset
 * of a plane within a buffer (-1 if the content does not include it). */
size_t qds_state_bytes(qds_handle h);
int32_t qds_row_pitch(qds_handle h);
int64_t qds_plane_offset(qds_handle h, int32_t plane);

/* Add a forward pulse of polarisation pol ('y','z': linear in mode 1; 'r','t':
 * radial / azimuthal in mode 0) to set 0 of buffer buf[cur].  f_K, f_J, f_G
 * are the real polarised field sampled at (x_i, r_{j+1/2}) [nr x nx],
 * (x_i, r_j) [(nr+1) x nx] and (x_i, r_{nr+1/2}) [nx], in device memory, float64. */
qds_status qds_add_pulse(qds_handle h, qds_state* st, int32_t pol, const double* f_K,
                         const double* f_J, const double* f_G, void* stream);

/* Advance n_steps steps (background set, axion, regenerated set).  With a
 * prescribed drive the library evaluates j_x^(0) of each step into a plane
 * of its own (allocated on the first such call, (nr+1) x row pitch elements),
 * which the fused kernels read as an extra current of mode 0.  The drive's
 * noise counter packs (step, lab column, row) as step << 32 | column << 12 |
 * row, so a call that would reach lab column 2^20 (nx - 1 + window, plus
 * n_steps with the moving window) fails with QDS_ESTATE. */
qds_status qds_step(qds_handle h, qds_state* fields, const qds_current* J, const qds_axion* axion,
                    int64_t n_steps, void* stream);

/* Options (synchronous, host only):
 *  QDS_OPT_PATH   QDS_PATH_AUTO (fused kernels when modes <= 8, and <= 4
 *                 for the moving window combined with the regenerated set,
 *                 which runs kernel AX),
 *                 QDS_PATH_STAGED (one kernel per stage), QDS_PATH_FUSED
 *  QDS_OPT_ROWS   radial rows per workgroup chunk of every fused kernel (1..4096)
 *  QDS_OPT_ROWS_A, QDS_OPT_ROWS_CUR, QDS_OPT_ROWS_B, QDS_OPT_ROWS_PAIR
 *                 the same for one kernel (background set, axion current,
 *                 regenerated set, two-step march), e.g. to replay heights
 *                 the tuner chose
 *  QDS_OPT_TUNE   1: the next qds_step of at least 8 steps on the fused path
 *                 times its first 8 steps (two passes over four tile heights
 *                 per kernel: 8, 16, 24, 32 for the background set with the
 *                 axion, 16, 24, 32, 48 for kernel AX, 8, 16, 26, 52 for the
 *                 background set alone, 4, 6, 8,
 *                 16 for the axion current, 16, 32, 52, 64 for the regenerated
 *                 set; HIP events around every launch) and keeps, for the
 *                 marches of the sets, the tallest height whose fastest trial
 *                 is within 2% of the fastest of all, for the axion current
 *                 the fastest (with QDS_OPT_PAIR in effect: its
 *                 first 8 pairs, the two-step march in place of kernel B);
 *                 the trial steps are ordinary
 *                 steps (the tiling changes no result).  Waits for the stream
 *                 once, after the trials.  Trials timed on a GPU that has
 *                 just been idle can mislead (its clocks still ramping): run
 *                 a few steps first.
 *  QDS_OPT_PRODUCTS QDS_PRODUCTS_DIRECT (default): the mode products of the
 *                 axion source and current by the direct convolution C_m
 *                 (Eq. mode_convolution); QDS_PRODUCTS_THETA: by a transform
 *                 pair through a theta grid of 3*modes - 2 points, exact for
 *                 modes 0..modes-1 (Sec. 3.3), on the staged kernels (the
 *                 handle then runs the staged path)
 *  QDS_OPT_OVERLAP 1: with the regenerated set on the fused kernels (kernel
 *                 A and the axion kernel, no prescribed drive), kernel A of
 *                 step k+1 runs on a second
 *                 stream of the handle beside kernel B of step k (they share
 *                 no plane); events order it after the axion kernel of step
 *                 k, and every launch is joined back into the caller's
 *                 stream before qds_step returns; steps are then single (it
 *                 takes precedence over QDS_OPT_PAIR).  0: one stream.
 *  QDS_OPT_KERNEL_AX 1: with the regenerated set on the fused kernels (up
 *                 to 4 modes; always with the moving window), one launch
 *                 (kernel AX) advances the
 *                 background set, forms the axion source, advances the axion
 *                 and forms the axion current from one read of the background
 *                 set and the axion (Sec. 2.1, Sec. 2.2 and Eqs. jax_mode,
 *                 jar_mode, jat_mode: 48 plane passes per step with kernel B
 *                 instead of 61), tile height QDS_OPT_ROWS_A (tuner
 *                 candidates 16, 24, 32, 48).  0 (default): kernel A writes
 *                 the axion source to scratch and the marched axion kernel
 *                 re-reads the background set to advance the axion and form
 *                 its current (measured faster on MI355X: the one-pass march
 *                 holds both windows, which halves its occupancy).
 *  QDS_OPT_PAIR   1: qds_step advances steps two at a time where the
 *                 two-step march applies (fused kernels; with the regenerated
 *                 set on kernel A and the marched axion kernel, without the
 *                 moving window or a prescribed drive; or the background set
 *                 alone without the axion, also with the moving window and
 *                 the drive, whose plane is then filled for both steps): one
 *                 launch marches one set through two
 *                 steps, the first step's rows handed to the second through
 *                 LDS, so the set's planes are read and written once per two
 *                 steps (temporal blocking of the Maxwell update of Sec. 2.1;
 *                 the results equal those of single steps bit for bit).  With
 *                 the regenerated set, kernel A and the axion kernel of the
 *                 first step write to a state-sized buffer of the handle
 *                 (allocated on first use, with 3 planes for the second
 *                 step's axion current), those of the second step into the
 *                 caller's other buffer.  Each pair flips fields->cur once and
 *                 adds 2 to fields->step; an odd last step is a single step.
 *                 Tile height QDS_OPT_ROWS_PAIR (default: two chunks; tuner
 *                 candidates 20 and the heights at which the launch's
 *                 workgroups just fill one, two, three, ... rounds of the
 *                 workgroups the GPU holds at once, the three smallest
 *                 distinct chunk counts; the timing slot of the march is that of
 *                 the set it advances, one launch per two steps.  1 is the
 *                 default; 0: single steps.
 *  QDS_OPT_PAIR_A 1: in pairs with the regenerated set (up to 4 modes, its
 *                 LDS within 160 KiB: 3 modes in FP64, 4 in FP32), the
 *                 background set is advanced by its own two-step march with
 *                 the axion source of both steps (2 x modes waves per tile,
 *                 the first step's field planes and the second S_a to the
 *                 pair buffer) in place of kernel A twice; tile height
 *                 QDS_OPT_ROWS_A (tuner candidates 16, 24, 32, 43).  The
 *                 results equal single steps bit for bit.  0 (default): kernel
 *                 A twice (measured faster on MI355X: the march's 2 x modes
 *                 waves in lockstep, one workgroup per CU in FP64).
 *  QDS_OPT_TIMING 1: qds_step brackets each kernel launch with a pair of HIP
 *                 events recorded on the caller's stream (no synchronisation;
 *                 the library keeps one pair per launch until reset); any
 *                 value resets the recorded launches */
enum {
    QDS_OPT_PATH = 1, QDS_OPT_ROWS = 2, QDS_OPT_TIMING = 3, QDS_OPT_TUNE = 4,
    QDS_OPT_ROWS_A = 5, QDS_OPT_ROWS_CUR = 6, QDS_OPT_ROWS_B = 7, QDS_OPT_PRODUCTS = 8, QDS_OPT_OVERLAP = 9,
    QDS_OPT_KERNEL_AX = 10, QDS_OPT_PAIR = 11, QDS_OPT_ROWS_PAIR = 12, QDS_OPT_PAIR_A = 13
};
enum { QDS_PRODUCTS_DIRECT = 0, QDS_PRODUCTS_THETA = 1 };
enum { QDS_PATH_AUTO = 0, QDS_PATH_STAGED = 1, QDS_PATH_FUSED = 2 };
qds_status qds_set_option(qds_handle h, int32_t key, int64_t value);

/* Summed kernel time (ms) and launch counts of the launches recorded since
 * timing was last set: index 0 = the background-set + axion kernel (kernel A;
 * the whole step on the staged path), index 1 = the regenerated-set kernel
 * (kernel B), index 2 = the axion-current kernel.  ms[3], launches[3].
 * Waits for the recorded events. */
qds_status qds_get_timing(qds_handle h, double* ms, int64_t* launches);

/* Tile heights (radial rows per workgroup) of the fused kernels in use:
 * rows[0] kernel A (or the background set without the axion), rows[1] the
 * axion current, rows[2] the regenerated set, rows[3] the two-step march;
 * *tuned = 1 once the autotuner (QDS_OPT_TUNE) has chosen them. */
qds_status qds_get_tiles(qds_handle h, int32_t* rows, int32_t* tuned);

/* 1 if qds_step runs the fused kernels for this handle. */
int32_t qds_uses_fused(qds_handle h);

/* Loss of the adjoint: the field energy of one mode of one set over the
 * columns x_begin <= i < x_end at the final step (E_x, B_x at t^{N-1/2}):
 *   L = w dx dr [ sum r_{j+1/2} (|T_r^+|^2 + |T_r^-|^2)/4 + sum r_j (|T_th^+|^2 + |T_th^-|^2)/4
 *               + sum r_j |E_x|^2/2 + sum r_{j+1/2} |B_x|^2/2 ],
 * w = 2 pi for mode 0 and pi otherwise (Eq. fourier_decomp), the axis row
 * weighted by dr/8 in place of r_0 (energy-centroid diagnostic of Sec. 4.1). */
typedef struct {
    int32_t set;       /* 0 background, 1 regenerated */
    int32_t mode;
    int32_t x_begin, x_end;
} qds_loss;

/* Bytes of the device pool qds_backward needs for n_steps with a checkpoint
 * every ckpt_every steps: ceil(n/C) checkpoints + (C+1) segment states + 2
 * adjoint states + 3 planes + 256 B. */
size_t qds_backward_pool_bytes(qds_handle h, int64_t n_steps, int64_t ckpt_every);

/* Gradient of the loss after n_steps steps from the state u0->buf[u0->cur]
 * with respect to that initial state, by the transposed (adjoint) step run
 * backward in time over recomputed states: the forward is checkpointed every
 * ckpt_every steps into ckpt_pool (caller-owned device memory of at least
 * qds_backward_pool_bytes), and each segment is recomputed before its
 * adjoint steps.  Gradients are over the real inner product Re sum conj(a) b
 * of the complex state.  Writes lambda0_out (a device buffer of
 * qds_state_bytes, same layout as a state), *loss_out (host) and, with the
 * regenerated set, dL_ds_out[2] (host): the sensitivities to the scales
 * s_phi of the Klein-Gordon source and s_j of the axion current.  u0 is not
 * modified.  Synchronises the stream before returning.  Not available for the
 * moving window, a prescribed drive or more than 4 modes (QDS_EUNSUPPORTED). */
qds_status qds_backward(qds_handle h, const qds_state* u0, const qds_current* J, const qds_axion* axion,
                        const qds_loss* loss, int64_t n_steps, int64_t ckpt_every, void* ckpt_pool,
                        size_t pool_bytes, void* lambda0_out, double* dL_ds_out, double* loss_out, void* stream);

/* Adds the loss of qds_backward evaluated on the state buffer buf to *out_dev
 * (a device double) and writes its gradient dL/du into grad_buf (a state
 * buffer; entries outside the loss are left untouched), or into a temporary
 * stream-ordered allocation when grad_buf is NULL. */
qds_status qds_loss_eval(qds_handle h, const void* buf, const qds_loss* loss, double* out_dev, void* grad_buf,
                         void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the loss of qds_loss_eval
 * added to *out_dev (a device double) without its gradient and without any
 * allocation.  Each 64-column x 4-row tile of the loss window leaves a partial
 * sum in a static device array of 65536 doubles (512 KiB per GPU, held until
 * the process ends), which one more workgroup adds in a fixed order.  Fails
 * with QDS_EINVAL when ceil((x_end - x_begin)/64) * ceil((nr+1)/4) > 65536.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams without ordering) race; calls on one stream do not.
 * The array is looked up (hipGetSymbolAddress) on the first call on each
 * device, with that device current. */
qds_status qds_loss_eval_noalloc(qds_handle h, const void* buf, const qds_loss* loss, double* out_dev, void* stream);

/* Adds Re sum conj(a) b over two state buffers to *out_dev (a device double). */
qds_status qds_dot(qds_handle h, const void* a, const void* b, double* out_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Particles of the PIC coupling (Sec. 3.1): field gather (Eq.
 * particle_field_gather), relativistic Boris push (Eqs. boris_parameters,
 * boris_update) and the charge-conserving modal current deposition (Eqs.
 * particle_deposition_path, particle_mode_weight, particle_modal_currents,
 * particle_azimuthal_current, face_current_x, face_current_r), which makes
 * the deposited current obey Eq. discrete_continuity in every retained mode.
 * Units: c = 1, momenta u = p/(m c), fields as in the state, charge-to-mass
 * ratio qm in code units (-1 for electrons), currents added to the planes in
 * the units of the field equations (d_t E = curl B - j).
 * --------------------------------------------------------------------------- */
typedef struct {
    double* x; double* y; double* z;       /* Cartesian positions at t^n (device, float64), updated to t^{n+1} */
    double* ux; double* uy; double* uz;    /* u at t^{n-1/2}, updated to t^{n+1/2} */
    const double* q;                       /* per-particle macro-charge Q_p (device), or NULL: ``charge`` each */
    int64_t count;
    double charge;
    double qm;
    int32_t clear;                         /* nonzero: zero the three current planes before depositing */
    int32_t pad_;
} qds_particles;

/* Advance every particle one step dt = dx in the fields of fields->buf[cur]
 * and add its current at t^{n+1/2} to three caller-owned planes (each
 * [modes][nr+1][row pitch] complex in the handle's dtype, the layout of a
 * state plane; cleared first when particles->clear): jx at (x_{i+1/2}, r_j) (half column i), jr at
 * (x_i, r_{j+1/2}) (row j), jt at (x_i, r_j).
 *  - Gather: transverse fields at t^n from T^n of the background set; E_x and
 *    B_x at t^{n-1/2}, or, with extrapolate != 0, extrapolated to t^n as
 *    3/2 F^{n-1/2} - 1/2 F^{n-3/2} with F^{n-3/2} from fields->buf[1 - cur]
 *    (the previous state after a qds_step).  The QDS B_x, B_r, B_theta are
 *    averaged along x onto x_i, x_{i+1/2}, x_{i+1/2} first.  Triangular shape
 *    (quadratic-spline weights on each grid); weights on rows below the axis
 *    go to the mirror row.
 *  - Push: Boris with dt = dx, then x^{n+1} = x^n + dt u^{n+1/2}/gamma.
 *  - Deposit: along x^n -> x^{n+1}; the angular current carries the path's
 *    angular displacement (j_theta = Q dtheta <g_x g_r>_m / (2 pi dx dr dt)),
 *    areas and volumes of the axis row with r_0 -> dr/8.
 * A particle whose old or new position leaves 2 <= x/dx <= nx - 3,
 * r/dr <= nr - 2 is left unchanged, deposits nothing and is counted in
 * *skipped_dev (a device counter, may be NULL).  Open x boundaries only
 * (QDS_EUNSUPPORTED otherwise).  Asynchronous on ``stream``.
 * Any particle order gives the same result to rounding; the step is fastest
 * with the particles sorted by cell in small 2D tiles, x fastest within a
 * tile (the planes' contiguous direction), e.g. 8 rows x 16 columns at two
 * particles per cell: each wave then gathers from a few cache lines per load,
 * and each workgroup of 256 deposits into an LDS tile over a compact box,
 * adding each tile value to the planes once. */
qds_status qds_particles_step(qds_handle h, const qds_state* fields, int32_t extrapolate, qds_particles* particles,
                              void* jx, void* jr, void* jt, unsigned long long* skipped_dev, void* stream);

qds_status qds_destroy(qds_handle h);

/* ---------------------------------------------------------------------------
 * Batched forward: many independent instances (each its own handle, grid,
 * mode count and state) advanced together.  Every step of the batch is one
 * launch per kernel class covering the tiles of all instances still running
 * (kernel A per mode count, the axion current per mode count, the
 * regenerated set), and up to graph_steps such steps are captured in one HIP
 * graph and launched as one.  When every instance has the regenerated set or
 * no axion at all (and QDS_OPT_PAIR is on for every handle), the steps run in
 * pairs as under qds_step: kernel A and the axion current twice (through each
 * handle's pair buffer), then the two-step march of each set, one launch per
 * class; an odd last step of a segment is a single step.  The update of each
 * instance is exactly that of qds_step on the fused kernels (Sec. 2 scheme
 * per instance), bit for bit.
 * --------------------------------------------------------------------------- */
typedef struct qds_batch_ctx* qds_batch;

/* Tile slots: radial rows per workgroup of each batched kernel class. */
enum {
    QDS_TILE_A1 = 0,        /* kernel A (background set + axion), 1..4 modes: slots 0..3 */
    QDS_TILE_CUR1 = 4,      /* axion current, 1..4 modes: slots 4..7 (rows per workgroup) */
    QDS_TILE_EM0 = 8,       /* background set without the axion */
    QDS_TILE_EM1 = 9,       /* regenerated set (kernel B) */
    QDS_TILE_PAIR0 = 10,    /* two-step march of the background set without the axion */
    QDS_TILE_PAIR1 = 11,    /* two-step march of the regenerated set */
    QDS_NTILES = 12
};

/* Groups ``count`` handles (1..4096, all distinct, one dtype, each able to
 * run the fused kernels: at most 4 modes, no moving window).  The handles
 * stay owned by the caller and must outlive the batch. */
qds_status qds_batch_create(const qds_handle* handles, int32_t count, qds_batch* out);

/* Advances instance k by n_steps[k] >= 0 steps.  states[count]: one state per
 * instance (caller-owned device buffers, updated: cur and step); J[count]:
 * per-instance currents (NULL = none; only the cold-plasma response, kind
 * QDS_J_NONE, is accepted); axion[count]: per-instance axion parameters (may
 * be NULL when no instance has the axion).  graph_steps >= 1 captures up to
 * that many steps per HIP graph (graphs are kept for replay while the set of
 * running instances is unchanged); 0 launches the kernels directly; -1
 * captures the whole uneven schedule of the call (every instance's steps,
 * the running set shrinking as instances finish) as one HIP graph and
 * launches it once (kept for replay while the tables, the tiles and the step
 * counts are the same).  With
 * tune != 0 and no tiles chosen yet, the autotuner times the first steps of
 * the run (two passes over the candidate tilings, 8 steps, or 8 pairs of
 * steps when the batch runs in pairs; only when every running instance has
 * that many steps left): each trial is an ordinary step (or pair) of the run,
 * and the tiling does not change any result.  Asynchronous on
 * ``stream``.  Graphs stay with the batch across calls and are replayed
 * whenever a call repeats a running set (or, with -1, a whole schedule) with
 * the same tiles: the argument table they read is rewritten in place, after
 * the previous call has finished, when the states or the physics change. */
qds_status qds_batch_run(qds_batch b, qds_state* states, const qds_current* J, const qds_axion* axion,
                         const int64_t* n_steps, int32_t graph_steps, int32_t tune, void* stream);

/* Tile heights in use (int32[QDS_NTILES]) and whether the autotuner chose them. */
qds_status qds_batch_get_tiles(qds_batch b, int32_t* tiles, int32_t* tuned);

/* Sets the tile heights (each 1..1024) and marks them as chosen. */
qds_status qds_batch_set_tiles(qds_batch b, const int32_t* tiles);

/* Launch counters since the batch was created (int64[4]): graph launches,
 * graphs instantiated, kernel launches issued outside graphs (graph_steps 0;
 * the autotuner's trial steps are not counted), and kernel launches carried
 * by the launched graphs. */
qds_status qds_batch_stats(qds_batch b, int64_t* stats);

const char* qds_batch_last_error(qds_batch b);

/* Waits for the batch's last run and releases its graphs and tables. */
qds_status qds_batch_destroy(qds_batch b);
const char* qds_last_error(qds_handle h);
const char* qds_version(void);

/* Measurement of the read + write bandwidth ceiling the marched kernels are
 * compared with: copies ``bytes`` (a multiple of 16) from src to dst, 16 bytes
 * per lane in a grid-stride loop over ``blocks`` workgroups of 256, with the
 * non-temporal (streaming) hint on loads and stores when streaming != 0.
 * QDS_EINVAL for null pointers, a size not a multiple of 16 or blocks < 1. */
qds_status qds_stream_copy(void* dst, const void* src, size_t bytes, int32_t streaming, int32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif
#endif
