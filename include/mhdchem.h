/*
 * mhdchem: one operator-split time step of ideal MHD with H/H2 chemistry on a
 * uniform periodic 3D grid, after Kulikov, Chernykh & Protasov (arXiv:1608.08748),
 * on one AMD MI355X (gfx950).
 *
 * The step (Sec. 2, the stages of the paper's list; heating/cooling, self-
 * gravity and the ionisation network are options of mhd_params):
 *   NONADV  pressure, Lorentz force and p dV work by a linearised Riemann
 *           problem with local-parabola data at every face (Sec. 2.1, 2.4),
 *           with the face-centred magnetic field updated from edge electric
 *           fields inside the same Runge-Kutta stage (Sec. 2.5);
 *   ADV     advection of rho, momentum, total and internal energy and H2
 *           density by upwind parabola averages (Sec. 2.6);
 *           each of the two stages is one three-stage SSP Runge-Kutta pass
 *           (Sec. 2.2);
 *   CHEM    semi-implicit H/H2 update per cell, reactions 1-4 (Sec. 2.7 and
 *           the rate appendix; with the ionisation network also H+ by
 *           reactions 5-8, Sec. 4.3), always in FP64;
 *   COOL    (option) explicit heating/cooling source (Sec. 2 stage 5,
 *           Sec. 2.8), FP64;
 *   REG     dual-energy regularisation (Sec. 2.8), always in FP64;
 *   GRAV    (option) Poisson stage with the 27-point Green's function
 *           (Sec. 2.9) and the gravity sources in NONADV.
 * The time step follows the CFL rule of Sec. 2.3.
 *
 * State (conserved, structure of arrays, x fastest, field order):
 *   0 rho  1 mx  2 my  3 mz  4 E (total energy density incl. B^2/2)
 *   5 e (internal energy density)  6 bx  7 by  8 bz  9 h2 (H2 mass density)
 * bx[i,j,k] is B_x on the lower x face (i-1/2, j, k) of cell (i,j,k); by and bz
 * likewise on the lower y and z faces.  Heaviside-Lorentz units (B^2/2 is the
 * magnetic pressure).  Cells are cubes of edge h = 1 / n[0].
 *
 * Conventions for every entry point:
 *   - return MHD_OK (0) or a negative status; no exception crosses the ABI;
 *   - host buffers are owned by the caller and only read/written during the
 *     call; device memory is the caller's workspace, borrowed for the box's
 *     lifetime and never freed by the library; nothing on the step path
 *     allocates device memory;
 *   - all device work goes to the caller's stream in submission order;
 *     mhd_step returns before the work finishes;
 *   - faults found on the device (non-finite or non-positive density or
 *     internal energy, a dt above the CFL bound) are latched in the workspace
 *     and returned by the next synchronising call (mhd_cfl_dt,
 *     mhd_conserved_totals, mhd_get_state) and stay latched until the next
 *     mhd_init_state / mhd_set_state;
 *   - one box is driven by one host thread at a time; distinct boxes are
 *     independent.
 */
#ifndef MHDCHEM_H
#define MHDCHEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MHD_OK = 0,
    MHD_EINVAL = -1,     /* bad argument (dims, NULL, dt not finite or <= 0, ...) */
    MHD_ENOMEM = -2,     /* workspace missing or smaller than mhd_workspace_bytes */
    MHD_EDEVICE = -3,    /* a HIP runtime call failed                             */
    MHD_ECFL = -4,       /* a step used dt above the CFL bound of its start state */
    MHD_ENONPHYS = -5,   /* non-finite or non-positive rho or e after a step       */
    MHD_ETOOLARGE = -6   /* box beyond the static scratch of an allocation-free    */
                         /* entry point (MHD_NOALLOC_MAX_CELLS)                    */
};

enum { MHD_FP64 = 0, MHD_FP32_MIXED = 1 };

/* Conserved fields of the state (host order): rho, mx, my, mz, E, e (= rho eps),
 * bx, by, bz (face values), h2 (= rho_H2), hp (= rho_H+, zero and untouched
 * unless the ionisation network is on); primitive fields for mhd_init_state:
 * rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2, x_hp. */
enum { MHD_NFIELDS = 11, MHD_NPRIM = 10 };

/* Stage selectors of mhd_debug_stage. */
enum {
    MHD_STAGE_NONADV = 1,    /* the NONADV Runge-Kutta stage only                   */
    MHD_STAGE_ADV = 2,       /* the ADV Runge-Kutta stage only                      */
    MHD_STAGE_TAIL = 3,      /* H2 clamp, chemistry and heating/cooling (if         */
                             /* enabled), regularisation                            */
    MHD_STAGE_NONADV_RHS = 4,/* one NONADV substage from the current state: writes  */
                             /* tau R(U) into the state slots (rho, h2 slots zero)  */
    MHD_STAGE_ADV_RHS = 5    /* one ADV substage: tau R(U) (face-field slots zero)  */
};

typedef struct {
    int32_t n[3];            /* cells along x, y, z (periodic); each >= 1, product < 2^31 */
    double gamma;            /* adiabatic index (5/3 in the configurations)             */
    double cfl;              /* Courant number of Sec. 2.3 (paper 0.2)                  */
    int32_t precision;       /* MHD_FP64 or MHD_FP32_MIXED (FP32 state and fluxes;      */
                             /* chemistry, regularisation, CFL and totals in FP64)      */
    double theta;            /* time coupling of the parabola averages: width           */
                             /* theta*|lambda|*tau (1 = the paper, 0 = edge values)     */
    int32_t chemistry;       /* 0 or 1                                                   */
    int32_t cooling;         /* 0 or 1: subgrid heating/cooling stage (Sec. 2 stage 5,  */
                             /* Sec. 2.8) after chemistry: explicit Euler step of        */
                             /* d(rho eps)/dt = d(rho E)/dt = Gamma - Lambda with the     */
                             /* appendix heating/cooling of reactions 1-4, FP64, energy  */
                             /* unit n_unit k_B T_unit, floor at 10 K                     */
    int32_t ionisation;      /* 0 or 1: ionisation network (Sec. 4.3, reactions 5-8):  */
                             /* H+ density advected as the 11th field, n_e = n_H+, its   */
                             /* semi-implicit update with chemistry, cosmic-ray heating  */
                             /* and collisional-ionisation cooling with heating/cooling, */
                             /* and gamma_eff = (5 n_H + 5 n_e + 7 n_H2) /               */
                             /* (3 n_H + 3 n_e + 5 n_H2) per cell in place of gamma      */
    double grav_G;           /* self-gravity (Sec. 2 equations, Sec. 2.9): gravitational  */
                             /* constant in code units, 0 = off.  When > 0 every step     */
                             /* solves Laplace(Phi) = 4 pi G rho with the 27-point        */
                             /* stencil in harmonic space (on-device FFT, zero-mean Phi)  */
                             /* and NONADV adds -rho grad(Phi) to m and -m.grad(Phi) to E */
                             /* (central differences).  Each n[d] must then be a power    */
                             /* of two, at most 1024 (else MHD_EINVAL).                   */
    double n_unit_cm3;       /* H nuclei per cm^3 per unit code density                 */
    double T_unit_K;         /* T = T_unit_K * mu * p / rho, mu = 1/(1 - x_H2/2)         */
    double t_unit_s;         /* seconds per code time unit                               */
    void *stream;            /* hipStream_t of the caller; NULL = the null stream       */
    void *workspace;         /* device memory, >= mhd_workspace_bytes, 256-byte aligned */
    size_t workspace_bytes;
} mhd_params;

typedef struct mhd_box mhd_box;

/* Device bytes the box needs for these parameters (three copies of the state
 * for the Runge-Kutta stages, face scratch, reduction partials and flags).
 * Host-only; returns 0 for invalid parameters. */
size_t mhd_workspace_bytes(const mhd_params *p);

/* Validate parameters and bind a box to the caller's workspace and stream.
 * Host-only (no device call).  *out is owned by the caller until mhd_destroy. */
int mhd_create(const mhd_params *p, mhd_box **out);

/* Load a primitive state: host FP64, MHD_NPRIM = 10 fields of n[0]*n[1]*n[2]
 * values, order rho, vx, vy, vz, p, bx_face, by_face, bz_face, x_h2, x_hp (H2
 * and H+ mass fractions).  Converts to conserved form on the device (Sec. 2:
 * rho E = e + rho v^2/2 + B^2/2 with cell-centre B the mean of the two faces,
 * p = (gamma-1) e, gamma_eff of the cell with the ionisation network),
 * computes the first CFL step, clears latched faults.  Synchronises. */
int mhd_init_state(mhd_box *b, const double *prim);

/* Load a conserved state (host FP64, the MHD_NFIELDS fields above); clears faults and
 * recomputes the CFL step.  Synchronises.  With mhd_get_state this is the
 * checkpoint / resume pair (bitwise for MHD_FP64). */
int mhd_set_state(mhd_box *b, const double *cons);

/* Copy the current conserved state to host FP64 (MHD_NFIELDS fields).  Synchronises;
 * returns a latched fault if any. */
int mhd_get_state(mhd_box *b, double *cons_out);

/* Gravitational potential of the current density (Sec. 2.9: the Poisson
 * stage run on the device), copied to phi_out: host FP64, nx*ny*nz values,
 * x fastest, zero mean.  Synchronises.  MHD_EINVAL if the box has no
 * self-gravity (grav_G == 0). */
int mhd_get_potential(mhd_box *b, double *phi_out);

/* CFL time step of the current state (Sec. 2.3): min over cells of
 * cfl*h / (|v| + b + c + c_a + c_s + c_f), b = |B|/sqrt(rho), c_a from B_x.
 * Synchronises; returns a latched fault if any. */
int mhd_cfl_dt(mhd_box *b, double *dt_out);

/* Advance the state by dt: NONADV, ADV, H2 clamp to [0, rho], chemistry,
 * heating/cooling (if enabled), regularisation; then the CFL step of the new state is computed on the
 * device.  Asynchronous.  dt must be finite and > 0 (else MHD_EINVAL); a dt
 * above the CFL bound of the start state (relative slack 1e-12 for MHD_FP64,
 * 1e-4 for MHD_FP32_MIXED, whose bound comes from FP32 values) latches
 * MHD_ECFL. */
int mhd_step(mhd_box *b, double dt);

/* As mhd_step with the device-resident CFL step of the current state
 * (no host round trip). */
int mhd_step_cfl(mhd_box *b);

/* FP64 sums over all cells of the MHD_NFIELDS conserved fields (field order above;
 * the face fields sum their face values).  Fixed-order tree reduction:
 * repeatable bit for bit.  Synchronises; returns a latched fault if any. */
int mhd_conserved_totals(mhd_box *b, double out[MHD_NFIELDS]);

/* For callers that cannot allocate device memory or bind a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the FP64 totals of mhd_conserved_totals (same kernels, same
 * fixed-order tree, so the same bits for the same stored values) of a state
 * held in the caller's own device memory.  Allocates nothing: the per-block
 * partial sums live in a static device array of the library (5.5 MiB per
 * device, held until the process ends).
 *   state      device pointer: MHD_NFIELDS fields of n[0]*n[1]*n[2] values,
 *              field order and layout of the box state (structure of arrays,
 *              x fastest), double for MHD_FP64, float for MHD_FP32_MIXED;
 *              only read
 *   precision  MHD_FP64 or MHD_FP32_MIXED
 *   n          cells along x, y, z; n[0]*n[1]*n[2] <= MHD_NOALLOC_MAX_CELLS
 *              (else MHD_ETOOLARGE, nothing launched)
 *   stream     hipStream_t of the current device; NULL = the null stream
 *   out        device pointer to MHD_NFIELDS doubles, written by the last
 *              kernel
 * Runs on the current device; asynchronous on stream (no synchronisation,
 * no host copy), so it can be captured.  Every call on one device shares
 * that device's partial-sum array: calls that overlap in time on one device
 * (on different streams or from different threads) race; calls ordered on
 * one stream do not.  Every partial is written before it is read, so no call
 * depends on what an earlier call left there.  The first call on a device
 * looks the array's device address up (hipGetSymbolAddress); MHD_EDEVICE if
 * that or a launch fails. */
enum { MHD_NOALLOC_MAX_CELLS = 16777216 };   /* 256^3 */
int mhd_conserved_totals_noalloc(const void *state, int32_t precision, const int32_t n[3], void *stream,
                                 double *out);

/* Run one part of the step on the current state (stage selectors above),
 * for per-stage parity checks.  Asynchronous. */
int mhd_debug_stage(mhd_box *b, int stage, double dt);

/* Kernel classes timed by mhd_set_timing / mhd_get_timing. */
enum {
    MHD_K_SETUP = 0,         /* state set-up (init_state, set_state); the step has no
                              * primitive pass: the NONADV face kernels form the
                              * primitives they read from the conserved state */
    MHD_K_NONADV_FACE = 1,   /* NONADV face Riemann solve (per axis)  */
    MHD_K_NONADV_UPDATE = 2, /* NONADV flux/CT update + RK            */
    MHD_K_ADV_FACE = 3,      /* ADV face fluxes (per axis)            */
    MHD_K_ADV_UPDATE = 4,    /* ADV update + RK                       */
    MHD_K_TAIL = 5,          /* clamp, chemistry, heating/cooling, regularisation, CFL */
    MHD_K_REDUCE = 6,        /* CFL / totals reductions               */
    MHD_K_POISSON = 7,       /* self-gravity: FFT Poisson solve       */
    MHD_NKCLASS = 8
};

/* Enable (1) or disable (0) per-launch HIP-event timing of the step's
 * kernels on the box's stream; enabling clears the accumulators.  Steps stay
 * asynchronous: the events of up to 1024 launches are held, and a step waits
 * for the recorded ones only once 512 are pending (about every 20 steps);
 * mhd_get_timing waits for all of them. */
int mhd_set_timing(mhd_box *b, int enable);

/* Accumulated device time (ms) and launch count per kernel class since
 * timing was enabled.  ms and counts have MHD_NKCLASS entries. */
int mhd_get_timing(mhd_box *b, double *ms, int64_t *counts);

/* Release the box (not the workspace, not the stream). */
int mhd_destroy(mhd_box *b);

const char *mhd_strerror(int status);

/* ------------------------------------------------------------------ */
/* Serving: many independent periodic boxes of uneven size share one GPU.
 * Requests are admitted in arrival order as slots and workspace memory free
 * up (the caller's workspace is the HBM budget; every box lives inside it),
 * their state stays resident in HBM, and each call of mhd_server_progress
 * advances every box in flight by one step of its own CFL dt with one merged
 * launch per kernel of the step program for all boxes (persistent: a resident
 * grid walks the union of the boxes' tiles).  A box computes
 * exactly the same bits alone or in any mix (same kernels, same per-box block
 * decomposition and reductions).  Boxes use the server's physics parameters;
 * n[0] <= 256.  Latencies are host wall-clock seconds since
 * mhd_server_create. */

typedef struct {
    int32_t precision;       /* MHD_FP64 or MHD_FP32_MIXED                       */
    double gamma, cfl, theta;
    int32_t chemistry;
    int32_t cooling;         /* as in mhd_params                                  */
    double n_unit_cm3, T_unit_K, t_unit_s;
    int32_t max_slots;       /* boxes in flight at most, 1..1024                 */
    void *stream;            /* hipStream_t; NULL = the null stream             */
    void *workspace;         /* device memory, 256-byte aligned: the HBM budget */
    size_t workspace_bytes;  /* (mhd_server_reserved_bytes of it hold the launch */
                             /* tables, the rest is the box pool)                */
    int32_t persistent;      /* 0: each merged launch takes one workgroup per    */
                             /*    tile of the union of the boxes' tiles;        */
                             /* 1: persistent launches: the grid is what the    */
                             /*    chip holds at once and each workgroup walks   */
                             /*    the tile list (same tiles, same bits)         */
    int32_t max_workgroups;  /* persistent launches: at most this many          */
                             /*    workgroups per launch (0: no cap beyond what  */
                             /*    the chip holds), e.g. to leave compute units  */
                             /*    to other work on the device                   */
} mhd_server_params;

typedef struct {
    int32_t n[3];            /* box cells along x, y, z                          */
    int32_t steps;           /* steps to run                                      */
    int32_t keep_state;      /* 1: keep the final conserved state for           */
                             /*    mhd_server_result                              */
    int32_t borrow;          /* 0: the primitive state is copied at submission;  */
                             /* 1: it is read in place when the request is       */
                             /*    admitted: the caller keeps it valid and       */
                             /*    unchanged until mhd_server_poll has returned  */
                             /*    the request's completion (no host copy; from  */
                             /*    pinned host memory the upload is one DMA)     */
} mhd_request;

typedef struct {
    uint64_t id;
    int32_t status;          /* MHD_OK or the box's latched fault                */
    int32_t steps;           /* steps run                                         */
    double t_submit, t_admit, t_done;   /* seconds since mhd_server_create       */
    double totals[MHD_NFIELDS]; /* conserved totals of the final state (FP64)   */
    int64_t cells;
    size_t bytes;            /* workspace bytes the box held                     */
} mhd_completion;

typedef struct mhd_server mhd_server;

/* Workspace bytes a server keeps for its launch tables. */
size_t mhd_server_reserved_bytes(void);

/* Pool bytes one box of n cells takes (0 for invalid input). */
size_t mhd_server_box_bytes(const mhd_server_params *p, const int32_t n[3]);

/* Create a server on the caller's workspace and stream (pins a 64 MiB host
 * staging buffer for the launch tables of two consecutive rounds and the
 * finished boxes' totals). */
int mhd_server_create(const mhd_server_params *p, mhd_server **out);

/* Queue a request with its primitive initial state (host FP64, the
 * mhd_init_state layout; copied, or borrowed with r->borrow = 1).  MHD_ENOMEM
 * if the box can never fit the pool, MHD_EINVAL for bad sizes or flags.  Does
 * not touch the device. */
int mhd_server_submit(mhd_server *s, const mhd_request *r, const double *prim, uint64_t *id);

/* One round: admit queued requests while a slot and pool memory are free
 * (first come, first served), launch one merged step of every box in flight,
 * then wait for the round launched by the previous call and report the boxes
 * that finished in it (mhd_server_poll).  Rounds are pipelined: the host work
 * of a call overlaps the previous round on the device, and a box's completion
 * is reported by the call after the one that launched its last step (keep
 * calling while requests are outstanding).  A finished box's memory returns to
 * the pool when its last step is launched (with keep_state, once its state is
 * copied out).  Outputs the numbers of boxes still stepping and of queued
 * requests. */
int mhd_server_progress(mhd_server *s, int *n_active, int *n_pending);

/* Take up to cap completion records (oldest first). */
int mhd_server_poll(mhd_server *s, mhd_completion *out, int cap, int *n);

/* Copy the final conserved state (MHD_NFIELDS fields, host FP64) of a finished request
 * submitted with keep_state = 1; count must be MHD_NFIELDS * cells.  Once per request. */
int mhd_server_result(mhd_server *s, uint64_t id, double *cons_out, size_t count);

/* Pool bytes in use now, the peak so far, and the pool size. */
int mhd_server_memory(mhd_server *s, size_t *used, size_t *peak, size_t *capacity);

/* Wait for the stream and release the server (not the workspace). */
int mhd_server_destroy(mhd_server *s);

#ifdef __cplusplus
}
#endif

#endif
