/*
 * pic.h -- C ABI of libpic, the MI355X (gfx950) hot path of a fully
 * relativistic electromagnetic particle-in-cell step.
 *
 * Method: Song, Wang & Li, "YUNIC: A Multi-Dimensional Particle-In-Cell Code
 * for Laser-Plasma Interaction", arXiv:2104.00642:
 *   - field solver: Yee staggered grid, leapfrog FDTD (Sec. II.B, Eqs. 9-10),
 *     applied as two half updates per step so that fields and particles exist
 *     at the same times (Sec. II.F);
 *   - particle pusher: Boris (Sec. II.C, Eqs. 11-16);
 *   - field interpolation with cell-integrated shape weights (Sec. II.D,
 *     Eqs. 17-19), the same shape for gather and deposit (Sec. II.E);
 *   - Esirkepov charge-conserving current deposit (Sec. II.E, Eqs. 20-22);
 *   - Monte-Carlo nonlinear Compton / Breit-Wheeler (Sec. IV, Eqs. 23-24).
 *
 * UNITS.  Every argument is in the normalized units of Sec. II.A (Eq. 8):
 * time in 1/w_r, length in c/w_r, E and B in m_e c w_r / e, momentum
 * u = p/m in units of c, charge in e, mass in m_e, density and macro-particle
 * weight in n_r = m_e w_r^2 / (4 pi e^2), current in c e n_r.  Then
 * dE/dt = curl B - J and div E = rho.
 *
 * GRID AND FIELD LAYOUT (device memory, caller-owned).  One plane per field
 * component, n[0]*n[1]*n[2] elements, element (i,j,k) at i + n0*(j + n1*k),
 * no guard cells, periodic in every axis.  Yee stagger (array index i of a
 * component staggered along an axis sits at (i + 1/2) * d):
 *   E_x, J_x: (1/2,0,0)  E_y, J_y: (0,1/2,0)  E_z, J_z: (0,0,1/2)
 *   B_x: (0,1/2,1/2)     B_y: (1/2,0,1/2)     B_z: (1/2,1/2,0)
 * In 2D3V (dim 2) n[2] = 1, the z offsets are dropped and d/dz = 0.
 * Field element type: float (PIC_FP32_MIXED) or double (PIC_FP64_PLAIN).
 *
 * PARTICLES (device memory, caller-owned, structure of arrays).
 *   PIC_FP32_MIXED: int32 packed cell index  cell = ix | iy << bx | iz << (bx+by)
 *     with bx = ceil(log2 n[0]), by = ceil(log2 n[1]) (pic_get_layout), float
 *     in-cell offsets off[a] in [0,1) (position x_a = (i_a + off_a) d_a), float
 *     momenta u[3], optional float weight w.
 *   PIC_FP64_PLAIN: double absolute positions x[a] in [0, n[a] d[a]), double
 *     momenta u[3], optional double weight w.
 * Positions and momenta are at the same full step n (Sec. II.F).
 *
 * STREAMS.  `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  Calls only enqueue work; they return before it finishes, and
 * none of them synchronizes the device.  Arrays must stay alive until the
 * stream is synchronized.  The context's scratch (straggler lists, sort
 * buffers, network outputs) is sized by pic_reserve; a call that needs more
 * allocates it then (hipMalloc, no synchronization) and keeps the outgrown
 * buffer until the next pic_reserve or pic_destroy.  Calls on different
 * streams share that scratch and must not overlap.
 *
 * ERRORS.  Argument and configuration errors are found before anything is
 * enqueued and returned as a pic_status with a message in pic_last_error().
 * HIP launch failures give PIC_E_HIP.  Data-dependent conditions seen by the
 * kernels set bits of a device status word read (and cleared) by pic_check().
 * Nothing aborts and no C++ exception crosses the ABI.  A context is not
 * thread-safe; several contexts may coexist.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_E_ARG = 1,          /* null or inconsistent argument                */
    PIC_E_CFL = 2,          /* dt above the Courant limit                   */
    PIC_E_UNSUPPORTED = 3,  /* order / dim / bc / precision not built       */
    PIC_E_NOMEM = 4,        /* device allocation of context scratch failed  */
    PIC_E_HIP = 5,          /* a HIP runtime call or launch failed          */
    PIC_E_CAPACITY = 6,     /* pic_check: particle creation hit capacity    */
    PIC_E_STATE = 7         /* pic_check: bad particle data was seen        */
} pic_status;

enum { PIC_FP32_MIXED = 0, PIC_FP64_PLAIN = 1 };
/* Boundaries, per axis.  Absorbing faces are built for x (bc[0]): the domain
 * is x in [0, (n[0]-1) d[0]] (the absorbing faces of the paper's 1D case,
 * Sec. III; their scheme is not printed).
 *   Fields: E_y, E_z on the two faces follow Mur's rule over each half step
 *   (G. Mur, IEEE Trans. EMC 23, 377 (1981)), at x = 0 acting on E - E_inc so
 *   that a pulse set by pic_set_laser enters; E_x, B_y, B_z half a cell
 *   beyond the far face stay 0.  PIC_BC_ABSORB: first order, a plane wave at
 *   angle theta from the normal comes back with amplitude
 *   (1 - cos theta)/(1 + cos theta).  PIC_BC_ABSORB2: second order (the
 *   transverse second differences of Engquist and Majda's condition), the
 *   square of that; it keeps the face values of the previous E half update in
 *   the context, so its first E half update after pic_init runs the
 *   first-order rule, and a context must not be switched between field sets.
 *   Particles: nothing is gathered from or deposited to x nodes beyond
 *   [0, n[0]), and a particle whose new position leaves the domain is
 *   absorbed: its weight is set to 0 (per-particle weights are required; it
 *   stays in the arrays, wrapped in x, until the caller drops it). */
enum { PIC_BC_PERIODIC = 0, PIC_BC_ABSORB = 1, PIC_BC_ABSORB2 = 2 };
/* Momentum update: Boris (Sec. II.C, Eqs. 13-16) or Vay, which Sec. II.C
 * names for fields whose electric and magnetic forces nearly cancel; Vay
 * solves u^{n+1} - u^n = q_m dt (E + (v^n + v^{n+1})/2 x B) in closed form
 * (J.-L. Vay, Phys. Plasmas 15, 056701 (2008)). */
enum { PIC_PUSH_BORIS = 0, PIC_PUSH_VAY = 1 };

/* Status-word bits reported by pic_check. */
enum {
    PIC_F_NONFINITE = 1u,   /* NaN/Inf momentum or offset on input           */
    PIC_F_OFFSET = 2u,      /* FP32 offset outside [0,1) or cell out of grid */
    PIC_F_STRAGGLER = 4u,   /* particle outside its tile window (handled by
                               the global-memory path; sort more often)      */
    PIC_F_CAPACITY = 8u,    /* QED creation beyond capacity (events dropped) */
    PIC_F_QED_SATURATED = 16u /* QED Method II acceptance above 1: the time step
                               is too long for the rate, events are missed   */
};

typedef struct {
    int32_t dim;            /* 2 = 2D3V, 3 = 3D3V                                     */
    int32_t order;          /* 1 = linear (CIC), 2 = quadratic, 4 = quartic (Sec. II.D) */
    int32_t precision;      /* PIC_FP32_MIXED or PIC_FP64_PLAIN                       */
    int32_t drift;          /* FP32 path: cells a particle may leave its tile between
                               sorts and still use the LDS window (0..4; default 2)  */
    int64_t n[3];           /* cells per axis; n[2] = 1 when dim = 2                  */
    double d[3];            /* cell sizes (c/w_r)                                     */
    double dt;              /* step (1/w_r); PIC_E_CFL unless dt*sqrt(sum 1/d^2) <= 1  */
    int32_t bc[3];          /* PIC_BC_PERIODIC; bc[0] may be PIC_BC_ABSORB(2)           */
    int32_t tile[3];        /* FP32 path tile in cells (must divide n); 0 = default   */
    uint64_t seed;          /* key of the counter-based generator (QED)               */
    double hbar_omega_mc2;  /* hbar w_r / (m_e c^2) for chi (2.4263e-6 at 1 um);
                               0 disables the chi output of the push                  */
    int32_t pusher;         /* PIC_PUSH_BORIS (0) or PIC_PUSH_VAY (1); PIC_E_ARG else  */
} pic_config;

typedef struct {
    double q;               /* charge (e)                                   */
    double m;               /* mass (m_e)                                   */
    double w0;              /* weight used when the particle w is NULL (n_r) */
} pic_species;

typedef struct {
    int64_t n;              /* live particles                                          */
    int32_t *cell;          /* FP32: packed cell                                       */
    float *off[3];          /* FP32: in-cell offsets                                   */
    double *x[3];           /* FP64: absolute positions                                */
    void *u[3];             /* float* (FP32) or double* (FP64)                         */
    void *w;                /* nullable; float* or double*                             */
    float *chi;             /* nullable; chi at step n+1/2 written by the push (FP32)  */
    int64_t *tile_start;    /* FP32 path: ntiles+1 offsets of the tile-sorted order,
                               written by pic_sort (dst) and read by the push and by
                               the next pic_sort of these arrays (src, as a hint)     */
    /* QED (pic_qed_step; NULL/0 otherwise) */
    double *tau;            /* optical depth accumulated since the last event         */
    float *tau_thr;         /* threshold -ln r of the next event                      */
    uint64_t *id;           /* unique identifiers (random streams, child identifiers) */
    int64_t capacity;       /* length of every array: particles created beyond it are
                               dropped and flagged PIC_F_CAPACITY                     */
    int64_t *n_dev;         /* device count: n plus the particles pic_qed_step created;
                               the caller reads it back and passes it as n next time  */
} pic_particles;

typedef struct {
    void *E[3];
    void *B[3];
    void *J[3];
} pic_fields;

/* Create a context for one grid and step (validates the configuration and
 * allocates the context's scratch).  Errors: PIC_E_ARG, PIC_E_CFL,
 * PIC_E_UNSUPPORTED, PIC_E_NOMEM, PIC_E_HIP; *out is NULL on error and
 * pic_last_error(NULL) holds the message.  FP32 path: the tile window,
 * tile + 2 drift + 5 cells per axis (tile + 2 drift + 7 with quartic
 * weights), takes 48 B per cell of LDS and must fit 159 KB (the 160 KB of
 * one workgroup less the push kernel's own 1 KB) and the grid, else
 * PIC_E_UNSUPPORTED. */
pic_status pic_init(const pic_config *cfg, void **out);
void pic_destroy(void *ctx);
const char *pic_last_error(const void *ctx);

/* Size the context's scratch for species of up to `particles` particles
 * (the push's straggler and bin lists, 12 B per particle; the sort's
 * buffers, 16 B per particle; with QED, the network outputs, 8 B per
 * particle), and free scratch outgrown since the last call.  A set-up call:
 * it synchronizes the device.  Errors: PIC_E_ARG (particles outside
 * [0, 2^31)), PIC_E_NOMEM. */
pic_status pic_reserve(void *ctx, int64_t particles);

/* Packed-cell layout and tiling chosen by pic_init: bits[3] per-axis field
 * widths of the packed cell, tile[3] tile size in cells, *ntiles number of
 * tiles (tile_start needs ntiles+1 entries). */
pic_status pic_get_layout(const void *ctx, int32_t bits[3], int32_t tile[3], int64_t *ntiles);

/*
 * Gather + Boris push + move + Esirkepov deposit for every particle of one
 * species (Secs. II.C-E), in the order of Sec. II.F:
 *   gamma = sqrt(1+|u|^2); x_h = x^n + dt u^n/(2 gamma)            (time n+1/2)
 *   E, B gathered at x_h with each component's staggered weights  (Eq. 19)
 *   Boris with gamma^{n+1/2} from u^-                              (Eqs. 13-16)
 *   v = u^{n+1}/gamma^{n+1}; x^{n+1} = x_h + dt v/2; deposit of the straight
 *   move x_h -> x_h + dt v (Eq. 12) into J                        (Eqs. 20-22)
 * fields->E, fields->B hold E^{n+1/2}, B^{n+1/2} (read only); fields->J is
 * ACCUMULATED into (the caller zeroes it once per step before the first
 * species).  Particles are updated in place and wrapped periodically.
 * FP32 path: particles must be in the order of the last pic_sort (tile_start
 * valid); particles that left their tile by more than `drift` cells, and
 * particles after tile_start[ntiles] (appended since the sort), are still
 * pushed correctly through global memory; stragglers are flagged
 * PIC_F_STRAGGLER and counted.  A particle whose offset is outside [0,1) or
 * whose packed cell is off the grid is flagged PIC_F_OFFSET and left
 * unchanged; NaN/Inf momenta or offsets are flagged PIC_F_NONFINITE.  The
 * context's straggler and bin lists hold up to n entries each (see
 * pic_reserve).  n = 0 is a no-op (the particle arrays
 * may then be NULL; the fields are still checked).
 * diag (nullable, device double[4]) receives += {sum w m (gamma^{n+1}-1) dV,
 * sum q w dV} in diag[0..1], computed in FP64 in a fixed order (diag[2] is
 * the field energy of pic_yee_step, diag[3] the Gauss residual of
 * pic_gauss_residual).  When chi is non-NULL
 * and hbar_omega_mc2 > 0 it receives chi_e of Sec. IV at the fields of x_h
 * and u^{n+1/2} = (u^n + u^{n+1})/2.
 */
pic_status pic_gather_push_deposit(void *ctx, const pic_species *sp, const pic_particles *p,
                                   const pic_fields *fields, double *diag, void *stream);

/*
 * Gather + push + deposit of several species (Secs. II.C-E, Sec. II.F: every
 * species of a step moves in the same fields and adds to the same J):
 * sp[k] and p[k] describe species k, nsp in [1, PIC_MAX_SPECIES], and each
 * species must be listed once.  The result is that of one
 * pic_gather_push_deposit per species in the order given, with one
 * difference: on the FP32 path the species share each tile's pass (its
 * field window is staged once and their currents meet in one fixed-point
 * window), so J is rounded to FP32 once per tile instead of once per tile
 * and species, and its last bits can differ.  Particle updates and flags
 * are the same bit for bit; diag receives the sums over the species.  The
 * FP64 plain path pushes the species one after another.  The call's scratch
 * (the per-species lists of pic_gather_push_deposit, for all species at
 * once) is grown on demand by the call itself, not by pic_reserve.  Errors
 * as pic_gather_push_deposit, and PIC_E_ARG for nsp out of range or a
 * species listed twice.
 */
#define PIC_MAX_SPECIES 4
pic_status pic_gather_push_deposit_multi(void *ctx, int32_t nsp, const pic_species *sp,
                                         const pic_particles *const *p, const pic_fields *fields,
                                         double *diag, void *stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pic_gather_push_deposit
 * with the same arguments, results and errors, but every scratch buffer of
 * the push (FP64 partials, straggler and bin lists, tile counters) taken
 * from a static device array of PIC_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; the call allocates nothing
 * and frees nothing.  Scratch per push (each part rounded up to 256 bytes):
 * FP32 path 12 B per particle, 52 B per tile, 4 KB and a counter; FP64 path 16 B per
 * 256 particles.  A push needing more returns PIC_E_ARG before anything is
 * enqueued (with 4096 tiles the FP32 path takes up to about 5.5e6
 * particles).  Every call on one GPU shares its array
 * and leaves its contents behind (what must start at zero is cleared by the
 * push's own kernels): calls that overlap in time on one GPU (other streams,
 * other threads, other contexts) race.
 */
#define PIC_NOALLOC_SCRATCH_BYTES (64ll << 20)
pic_status pic_gather_push_deposit_noalloc(void *ctx, const pic_species *sp, const pic_particles *p,
                                           const pic_fields *fields, double *diag, void *stream);

/*
 * Half field update (Sec. II.B Eqs. 9-10 split as in Sec. II.F):
 *   half = 1:  E += (dt/2)(curl B - J);  B -= (dt/2) curl E
 *   half = 2:  B -= (dt/2) curl E;       E += (dt/2)(curl B - J)
 * A step is half 1 (J = J^n), the particle push (J^{n+1}), half 2.
 * diag (nullable, device double[4]) receives diag[2] += 1/2 sum(E^2+B^2) dV
 * of the fields after the update (FP64, fixed order) when half = 2.
 */
pic_status pic_yee_step(void *ctx, int32_t half, const pic_fields *fields, double *diag,
                        void *stream);

/*
 * Tile binning (FP32 path).  Writes src's particles into dst in the order
 * (tile, rank of the particle among those of its cell in src order, key of
 * the cell within the tile), and dst->tile_start[0..ntiles] (first index of
 * each tile).  Tiles are tile[0] x tile[1] (x tile[2]) blocks of cells
 * numbered x-fastest.  Within a tile cells are grouped by the parities of
 * their tile-local coordinates, classes in the order 00 11 01 10 (2D) or
 * 000 111 001 110 010 101 100 011 ((x, y, z) parities), each class
 * z-, y-, x-slowest to fastest on the halved coordinates.  A particle
 * whose packed cell is off the grid (a field beyond its cell count, any bit
 * above y in 2D, a negative cell) has no tile: such particles follow the
 * last tile in src order, and tile_start[ntiles] is the number of particles
 * on the grid (the push then flags them PIC_F_OFFSET and leaves them
 * unchanged).  dst arrays must hold src->n elements and may not alias src.
 * Every non-NULL src array (cell, off, u, w, chi, tau, tau_thr, id) is
 * permuted into the matching dst array.  Bit-exact and deterministic.
 * src->tile_start (nullable, ntiles+1 entries, not dst->tile_start) is read
 * as a hint: the tile offsets of src's own order, as the sort that produced
 * src wrote them.  Particles still inside the segment of their tile keep
 * their relative order without being sorted again, so only the particles
 * that changed tiles since (and those appended after tile_start[ntiles])
 * pass through the key sort.  Any hint gives the same result: one that is
 * not non-decreasing within [0, src->n] is ignored on the device, and a
 * stale one only costs time.
 */
pic_status pic_sort(void *ctx, const pic_particles *src, const pic_particles *dst, void *stream);

/*
 * Monte-Carlo QED step (Sec. IV) on the FP32 particle layout: Method I in
 * optical-depth form (modes PIC_QED_TABLE, PIC_QED_MLP) or Method II
 * (PIC_QED_METHOD2).  Rates per unit time (1/w_r):
 *   W_rad  = alpha/(sqrt3 pi) (m c^2/hbar w_r) F_rad(chi_e) / gamma     (Eq. 23)
 *   W_pair = alpha/(sqrt3 pi) (m c^2/hbar w_r) F_pair(chi_g) / eps_gamma (Eq. 24)
 * Each particle carries tau (FP64) and tau_thr; tau += W dt.  When tau >=
 * tau_thr an event happens: the energy fraction comes from the inverse
 * cumulative spectrum at a uniform r, tau <- 0, tau_thr <- -ln r'.  With
 * (r, r') = Philox4x32-10(counter (id_lo, id_hi, step, 0), key seed) mapped to
 * (0,1) by 52 bits each.
 *   Leptons (chi from the last push): photon of energy u gamma along u,
 *     recoil u <- u (1 - eps_gamma/|u|) (clamped at 0); the photon is appended
 *     to `photons` when eps_gamma >= photon_min_energy.
 *   Photons (momentum k = eps_gamma k^, chi_gamma computed here at the fields
 *     of `fields` after moving dt at c and written to chi when chi is not
 *     NULL): above 2 m c^2 an event appends a positron with x eps_gamma and
 *     an electron with (1-x) eps_gamma along k and sets the photon weight to
 *     0.  Photons need per-particle weights (PIC_E_ARG otherwise), and in
 *     PIC_QED_MLP mode the chi array, where the network reads this step's
 *     chi_gamma.  With absorbing x faces a photon whose new position leaves
 *     [0, (n[0]-1) d[0]] is absorbed (weight 0, chi 0, no pair), and no
 *     field is gathered from x nodes beyond [0, n[0]).
 * Created particles: identifier Philox(counter (parent_lo, parent_hi, step,
 * 0x80000000 | tag), key seed) (tag 1 photon, 2 positron, 3 electron), tau 0,
 * tau_thr from the counter (id_lo, id_hi, step, 1); parent position and
 * weight.  F and the inverse spectra come from tables the library computes
 * with its own quadrature at pic_init (PIC_QED_TABLE), or from the trained
 * network (PIC_QED_MLP; chi outside the trained range, or within 0.1 decade
 * of its ends, uses the tables).
 * Requires hbar_omega_mc2 > 0.
 * Method II (rejection; the tau and tau_thr of existing particles are neither
 * read nor written): with
 * the same (r, r') = (r1, r2), the proposal is u0 = r1^3 (emission) or
 * x0 = r1 (pairs) and the event happens when
 *   3 r1^2 (d^2W_rad/du dt)(u0) dt > r2   or   (d^2W_pair/dx dt)(x0) dt > r2,
 * the paper's condition with the time step written in (x = eps_+/eps_gamma).
 * The densities come from tables of the normalized spectra the library
 * computes at pic_init (bilinear in log10 chi and in acos(1 - 2 sigma)).
 * Acceptances above 1 set PIC_F_QED_SATURATED (pic_check reports the flag;
 * the step still returns PIC_OK).  Photons and the kinematics are as in
 * Method I.
 */
enum { PIC_QED_TABLE = 0, PIC_QED_MLP = 1, PIC_QED_METHOD2 = 2 };
typedef struct {
    const pic_particles *electrons;   /* nullable */
    const pic_particles *positrons;   /* nullable */
    const pic_particles *photons;     /* nullable */
    const pic_fields *fields;         /* E, B at the end of the step (FP32)        */
    int32_t mode;                     /* PIC_QED_TABLE, PIC_QED_MLP, PIC_QED_METHOD2 */
    uint32_t step;                    /* step index: counter of the random streams  */
    double photon_min_energy;         /* m c^2 units                                */
    const void *mlp;                  /* PIC_QED_MLP: device network (layout below) */
} pic_qed_args;
pic_status pic_qed_step(void *ctx, const pic_qed_args *args, void *stream);

/*
 * Surrogate network of the QED module: 4 -> 64 -> 64 -> 2 perceptron,
 * h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3, BF16 weights,
 * FP32 biases, FP32 accumulation (BF16 matrix cores).  Each weight is a pair
 * of BF16 terms, hi = bf16(w) and lo = bf16(w - hi), and in the forward pass
 * each activation enters as two BF16 terms too (hi and remainder); products
 * take hi x hi + hi x lo + lo x hi.  Device layout (PIC_MLP_BYTES, row-major,
 * input index first): hi terms W1 bf16[4][64] @0, W2 bf16[64][64] @512,
 * W3 bf16[64][2] @8704; b1 f32[64] @8960, b2 f32[64] @9216, b3 f32[2] @9472;
 * lo terms W1 @9480, W2 @9992, W3 @18184.  Inputs x = ((log10 chi - c)/h, 2 rho(r) - 1, [emission],
 * [pairs]) where log10 chi spans [c-h, c+h] = [-4, 3] (emission) or
 * [-1.7, 3] (pairs) and rho(r) = 1 - sqrt(1-r) (emission) or
 * acos(1-2r)/pi (pairs); outputs y0 = ln(F_rad/chi) or ln F_pair + 8/(3 chi),
 * y1 = u^(1/3) (photon energy fraction) or x (positron fraction).
 * Training state (PIC_MLP_STATE_FLOATS floats, FP32): parameters, Adam first
 * and second moments and the gradient (PIC_MLP_NPARAM each, order W1, b1, W2,
 * b2, W3, b3), then the Adam step count.
 */
#define PIC_MLP_NPARAM 4610
#define PIC_MLP_BYTES 18440
#define PIC_MLP_OFF_W1 0
#define PIC_MLP_OFF_W2 512
#define PIC_MLP_OFF_W3 8704
#define PIC_MLP_OFF_B1 8960
#define PIC_MLP_OFF_B2 9216
#define PIC_MLP_OFF_B3 9472
#define PIC_MLP_OFF_W1_LO 9480
#define PIC_MLP_OFF_W2_LO 9992
#define PIC_MLP_OFF_W3_LO 18184
#define PIC_MLP_STATE_FLOATS (4 * PIC_MLP_NPARAM + 1)

/* y[n][2] = network(x[n][4]) (device arrays). */
pic_status pic_mlp_forward(void *ctx, const void *mlp, const float *x, int64_t n, float *y, void *stream);
/* grad[PIC_MLP_NPARAM] += d/dparams of sum_rows sum_o w_o (y_o - t_o)^2 / (2n),
 * w = (10, 1) (the rate output carries the accuracy target), with the
 * network's (BF16) weights; *loss (nullable) += that loss. */
pic_status pic_mlp_grad(void *ctx, const void *mlp, const float *x, const float *t, int64_t n, float *grad,
                        float *loss, void *stream);
/* `iters` Adam steps on consecutive batches of `batch` rows of (x, t),
 * starting from the state's parameters, with the step size decaying from lr
 * to 0 as 0.5 lr (1 + cos(pi it / iters)); the BF16 network is written to
 * mlp after every step; *loss (nullable) receives the last batch's loss. */
pic_status pic_mlp_train(void *ctx, float *state, void *mlp, const float *x, const float *t, int64_t n,
                         int32_t batch, int32_t iters, float lr, float *loss, void *stream);
/* n training rows from the library's tables (row i: process i & 1, log10 chi
 * and r uniform from Philox(counter (i_lo, i_hi, 0, 7), key seed)). */
pic_status pic_qed_training_data(void *ctx, int64_t n, uint64_t seed, float *x, float *t, void *stream);
/* Table queries: what = 0 F(chi) (r unused), 1 inverse spectrum at (chi, r);
 * proc 0 photon emission, 1 pair creation. */
pic_status pic_qed_table_lookup(void *ctx, int32_t proc, int32_t what, const float *chi, const float *r,
                                int64_t n, float *out, void *stream);

/*
 * Pulse injected through the x = 0 face (requires absorbing x faces), in
 * laser units (w_r = w_L: wavelength 2 pi, critical density 1):
 *   E_y = a0 exp(-r^2/waist^2) S((t - t0 - x)/duration) sin(x - t),
 *   E_z = the same with sin(x - t + pi/2) when circular, else 0,
 * S(s) = sin^2(pi s) on [0, 1], r from the box's transverse axis.  `t` sets
 * the library's field clock: the time of E and B at the next
 * pic_yee_step(half = 1); each half = 2 call advances it by dt.  a0 = 0
 * switches the pulse off.  Copies *laser.
 */
typedef struct {
    double a0;          /* peak field amplitude (m c w_r / e)           */
    double waist;       /* 1/e field radius (c/w_r)                      */
    double duration;    /* length of the sin^2 field envelope (1/w_r)    */
    double t0;          /* time the envelope starts entering at x = 0    */
    int32_t circular;   /* 0: E along y; 1: circular (a0 on E_y and E_z) */
} pic_laser;
pic_status pic_set_laser(void *ctx, const pic_laser *laser, double t);

/*
 * Charge density on the nodes (the integer-node shape weights of Sec. II.D):
 *   rho(i) += q w prod_a W(i_a - x_a/d_a)
 * for every particle of the species, at x^n (at_half = 0) or at the half
 * step x^n + dt u^n / (2 gamma^n) (at_half = 1: the positions of the
 * push's start point, the time of E after pic_yee_step(half = 1)).  rho is a
 * device double[n0 n1 n2] in the field layout, ACCUMULATED into (FP64
 * atomics), periodic on every axis.  Either particle layout.  n = 0 is a
 * no-op.  Errors: PIC_E_ARG.
 */
pic_status pic_deposit_rho(void *ctx, const pic_species *sp, const pic_particles *p, int32_t at_half,
                           double *rho, void *stream);

/*
 * Gauss residual (Sec. II.B: with a charge-conserving current, Eq. 5, the
 * divergence equations, Eqs. 1-2, keep holding as they held initially):
 *   residual(i) = sum_a (E_a(i) - E_a(i - e_a)) / d_a - rho(i)
 * on the nodes, in FP64 from the FP32 or FP64 E planes.  residual
 * (nullable, device double[n0 n1 n2]) receives it; diag (nullable, device
 * double[4]) receives diag[3] = max(diag[3], max_i |residual(i)|).  rho as
 * accumulated by pic_deposit_rho over the species.  Errors: PIC_E_ARG.
 */
pic_status pic_gauss_residual(void *ctx, const pic_fields *fields, const double *rho, double *residual,
                              double *diag, void *stream);

/*
 * Self-fields of a relativistic bi-Gaussian bunch (Sec. III(c): Poisson's
 * equation in the bunch's rest frame, then the Lorentz transformation to the
 * laboratory frame).  The bunch of particles of charge `charge` has the lab
 * density charge-carrier density n_b exp(-sum_a (x_a - center_a)^2 /
 * (2 sigma_a^2)) and moves along +x with Lorentz factor gamma.  In its rest
 * frame it is gamma sigma_x long; its field there is the free-space solution
 * of lap phi' = -rho' (div E = rho, the units of Eq. 8), and in the lab
 *   E_x = E'_x,  E_perp = gamma E'_perp,  B = beta x^ x E,
 * evaluated at x' = gamma (x - center_x) on every node at each component's
 * Yee position.  In a 2D box the bunch is uniform along z (sigma[2] and
 * center[2] unused; E_z and B_y stay as they are).  The fields are ADDED to
 * fields->E and fields->B (J untouched), in the context's precision, the
 * arithmetic in FP64.  Free space: no periodic images and no faces; the box
 * should hold the bunch well inside it.  Errors: PIC_E_ARG (NULL arguments,
 * gamma < 1, sigmas not > 0, non-finite values).
 */
typedef struct {
    double charge;      /* charge of the bunch's particles (units of e, with sign) */
    double density;     /* peak lab density n_b of those particles (units of n_r)  */
    double center[3];   /* centre (absolute position)                             */
    double sigma[3];    /* lab rms sizes                                          */
    double gamma;       /* Lorentz factor of the motion along +x (>= 1)           */
} pic_beam;
pic_status pic_beam_fields(void *ctx, const pic_beam *beam, const pic_fields *fields, void *stream);

/* Synchronize `stream`, return the device status word in *flags (nullable)
 * and the number of straggler particles since the last check in
 * *stragglers (nullable), then clear both.  Returns PIC_E_CAPACITY if
 * PIC_F_CAPACITY is set, else PIC_E_STATE if NONFINITE or OFFSET is set,
 * else PIC_OK. */
pic_status pic_check(void *ctx, void *stream, uint32_t *flags, uint64_t *stragglers);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
