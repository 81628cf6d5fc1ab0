/*
 * fuglbm.h -- C ABI of the MI355X (gfx950) implementation of the per-time-step
 * lattice update of the fugacity-based well-balanced multicomponent lattice
 * Boltzmann method (Soomro, Ayala, Peng & Ayala, arXiv:2212.10680).
 *
 * One step (Sec. III.B, steps 1-9) at every node of a periodic lattice:
 *   moments and velocity (step 1, with the force of the previous time step),
 *   molar densities and mole fractions (step 2), mixing rules (step 3,
 *   App. C eqs. eqmixingrulesaSRK/eqmixingrulesbm), EOS pressure (step 4,
 *   eqPREOS/eqSRKEOS/eqvdwEOS), ln f_i (step 5, eqfugupdatePR/SRK/VDW),
 *   interface potential mu_I,i = -sum_j sqrt(kappa_i kappa_j) lap(rho~_j)
 *   (step 6, eqChemPotI2/eqkappa/eq2ndder), component force
 *   F_i = -rho~_i RT grad ln f_i - rho~_i grad mu_I,i (step 7, eqforceFugLBM,
 *   eq1stder), well-balanced equilibrium and forcing (step 8, eqLBEMCb with
 *   rho_0 = 0 and eqLBEMCfinal3), collision and streaming (step 9, eqLBEMCa).
 *
 * Conventions
 *   - Lattice units; the caller passes the gas constant R (1 in lattice units).
 *   - Node index n = x + nx*(y + ny*z), x fastest; D2Q9 uses nz = 1.
 *   - Field arrays are host pointers, row-major [component or axis][node], and
 *     are owned by the caller; the library copies in and out.
 *   - Every call returns 0 (FL_OK) or a negative status; no exception crosses
 *     the ABI.  fl_last_error() gives a message for the last failure of a
 *     handle (HIP error text included for FL_EDEVICE).
 *   - A handle is used from one host thread at a time; there is no locking.
 *     All device work of a handle is issued on its HIP stream.
 */
#ifndef FUGLBM_H
#define FUGLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FL_OK 0
#define FL_EINVAL (-1)    /* invalid argument (see fl_create)                        */
#define FL_EDOMAIN (-2)   /* initial state outside the EOS domain: rho~_i <= 0,
                             rho~ b_m >= 1 or non-finite                               */
#define FL_ENOMEM (-3)    /* device or host allocation failed / buffer too small     */
#define FL_EDEVICE (-4)   /* HIP runtime error                                       */
#define FL_ENUMERIC (-5)  /* a step met a node outside the EOS domain (the scheme
                             went unstable); the state is not rolled back             */
#define FL_ENOTCONV (-6)  /* fl_run_until reached max_steps                          */
#define FL_EAGAIN (-7)    /* server cannot admit the request now                     */

#define FL_MAX_COMP 4

enum { FL_EOS_PR = 0, FL_EOS_SRK = 1, FL_EOS_VDW = 2 };
enum { FL_D2Q9 = 0, FL_D3Q19 = 1 };
enum { FL_BGK = 0, FL_MRT = 1 };
enum { FL_FP64 = 0, FL_FP32POP_FP64EOS = 1 };
enum { FL_FORCE_WB = 0, FL_FORCE_STANDARD = 1 };

/* One component (Sec. IV, Table tabCompProp; App. C): critical temperature and
 * pressure, acentric factor, molar mass M (step 2) and interface strength kappa
 * (eqs. eqChemPotI2, eqkappa). */
typedef struct fl_component {
    double Tc, Pc, omega, M, kappa;
} fl_component;

/* Problem statement.
 *   ncomp       1..FL_MAX_COMP
 *   comp        [ncomp] component constants; Tc, Pc, M > 0, kappa >= 0
 *   kij         [ncomp*ncomp] binary interaction coefficients delta_ij of
 *               eq. eqmixingrulesaSRK2, symmetric with zero diagonal; NULL = 0
 *   T, R        temperature and gas constant (R = 1 in lattice units)
 *   eos         FL_EOS_PR (App. C eqPREOS), FL_EOS_SRK, FL_EOS_VDW
 *   lattice     FL_D2Q9 (the paper's lattice) or FL_D3Q19 (same equations, D = 3)
 *   nx,ny,nz    periodic lattice; nz = 1 for D2Q9
 *   collision   FL_BGK (eq. eqLBEMCa) or FL_MRT: m = M g,
 *               m* = m - S (m - M g_eq) + (I - S/2) M F_a, with the orthogonal
 *               moment basis of Lallemand-Luo (D2Q9) / d'Humieres (D3Q19)
 *   tau         relaxation time, > 0.5
 *   mrt_rates   [4] = {s_j, s_nu, s_e, s_ghost}: component momentum, traceless
 *               stress, energy (trace) and all higher moments; NULL gives
 *               {1/tau, 1/tau, 1, 1}; ignored for BGK
 *   precision   FL_FP64: populations stored and collided in FP64.
 *               FL_FP32POP_FP64EOS: populations stored and collided in FP32 (the
 *               rest population as its offset from the initial density), EOS,
 *               logarithms, stencils and reductions in FP64
 *   force_time_level  0: the velocity of step 1 uses the previous step's force
 *               (as written in Sec. III.B, step 1); 1: this step's force
 *   force_model FL_FORCE_WB: well-balanced scheme (equilibrium eq. eqLBEMCb with
 *               rho_0 = 0, forcing eq. eqLBEMCfinal3, force eq. eqforceFugLBM);
 *               FL_FORCE_STANDARD: the standard-LBM form of Sec. V (force
 *               eq. eqForceGen = the fugacity force + c_s^2 grad rho_i, the
 *               standard equilibrium w_a rho_i (1 + e.u/c_s^2 + ...), Guo forcing
 *               without the grad rho_i terms); FP64 populations only
 *   stencil     FL_STENCIL_AXIS: the central differences of eq1stder and
 *               eq2ndder along the axes (the paper's); FL_STENCIL_ISOTROPIC:
 *               the lattice-weighted stencils grad f = (1/c_s^2) sum_a w_a e_a
 *               f(x + e_a), lap f = (2/c_s^2) sum_a w_a (f(x + e_a) - f(x)),
 *               equal to the axis ones on fields that vary along one axis and
 *               stable for 3-D droplets, where the axis ones are not.  With
 *               them a step is the moments pass and a z-marching collide pass
 *               that computes -lap(phi) itself where it fits (D3Q19, N_c <= 3,
 *               nx % 64 == 0, ny % 4 == 0, nz >= 2), otherwise three
 *               passes (moments, -lap(phi) at every node, one-thread-per-node
 *               collide); never
 *               the one-launch form; fl_required_bytes counts one more FP64
 *               field, and the batched server rejects them
 *               (FL_EINVAL) */
/* Stencils of the gradients and Laplacians of steps 6-7 (fl_params.stencil). */
#define FL_STENCIL_AXIS 0
#define FL_STENCIL_ISOTROPIC 1

typedef struct fl_params {
    int ncomp;
    const fl_component* comp;
    const double* kij;
    double T;
    double R;
    int eos;
    int lattice;
    int nx, ny, nz;
    int collision;
    double tau;
    const double* mrt_rates;
    int precision;
    int force_time_level;
    int force_model;
    int stencil;
} fl_params;

typedef struct fl_solver fl_solver;

/* Validate params; FL_EINVAL when ncomp is out of range, tau <= 0.5, a Tc, Pc or
 * M <= 0, a kappa < 0, kij not symmetric or with a non-zero diagonal, a
 * lattice dimension < 1 (or nz != 1 for D2Q9), N = nx*ny*nz >= 2^29,
 * N * ncomp * s >= 2^32 or N * D * s >= 2^32 with s = 8 for FP64 and 4 for
 * FP32 populations (every per-array byte offset, populations of one direction
 * and the force history of D values per node included, stays below 2^32), an
 * unknown enum, FL_FORCE_STANDARD with FP32 populations. */
int fl_validate(const fl_params* p);

/* Device bytes a solver needs for params (both population buffers, auxiliary
 * fields, reduction scratch).  Sets *bytes; FL_EINVAL on bad params. */
int fl_required_bytes(const fl_params* p, size_t* bytes);

/* Create a solver that allocates its own device memory and HIP stream on the
 * current device.  The populations start at zero: call fl_set_state next. */
int fl_create(const fl_params* p, fl_solver** out);

/* Create a solver on caller-owned device memory (>= fl_required_bytes bytes,
 * 256-byte aligned, e.g. a torch tensor) and a caller-owned hipStream_t (may be
 * NULL for the null stream).  The caller keeps both alive until fl_destroy. */
int fl_create_ext(const fl_params* p, void* device_mem, size_t bytes, void* hip_stream,
                  fl_solver** out);

/* Launch tuning (kernel variants, block sizes, visiting orders; none of them
 * changes a result bit).  spec = "key=value[,key=value...]" applied on top of
 * the measured defaults for the solver's lattice (each call starts from the
 * defaults; NULL or "" restores them).  Keys: k1block, k2block (threads per
 * block of the moments and the plain collide pass: 64, 128, 192, 256), remap
 * (XCD-contiguous block order of both passes, 0/1), remap2 (of the collide
 * pass only), nt (non-temporal population stores), fused (one-launch step on
 * D3Q19 lattices with ny >= 64 and nx % 16 == 0, axis stencils), zmarch
 * (z-marching collide pass where it fits: D3Q19, N_c <= 3, nx % 64 == 0,
 * ny % 4 == 0; with the isotropic stencils it also computes -lap(phi), so no
 * Laplacian pass runs), rev (the collide pass sweeps the nodes in the
 * reverse order), order (y-major rows inside per-XCD z-slabs), csplit (with
 * the isotropic stencils and N_c = 3: the z-marching collide pass gives each
 * component its own 256 threads, 1 by default; 0 keeps a node in one thread),
 * mpair (N_c >= 3, FP32 populations, an even node count, the moments pass at
 * its default 256-thread blocks in plain order: two consecutive nodes per
 * thread, 1 by default; 0 one node per thread; the same results either way),
 * zorder (block order of the z-marching collide passes: 0 XCD-contiguous
 * chunks, 1 XCD y-bands, all XCDs marching through the same planes; 1 by
 * default with the isotropic stencils and N_c >= 3), zlen (planes per z-marching workgroup, 1..4096), bands and lapbands (XCD-band order of
 * the plain collide pass and of the interface-Laplacian pass: the rows of each
 * plane cut into that many bands, a multiple of 8, each XCD sweeping its bands
 * along z; 0 = off).  FL_EINVAL (tuning unchanged) for an
 * unknown key or an out-of-range value.  Synchronises the solver's stream;
 * takes effect from the next step.  Nothing reads the environment. */
int fl_set_tuning(fl_solver* s, const char* spec);

void fl_destroy(fl_solver* s);
const char* fl_last_error(const fl_solver* s);
const char* fl_status_string(int status);

/* Lattice table used by fl_get_populations: velocities e[Q][3] (z = 0 for
 * D2Q9) and weights w[Q]; *q receives Q.  Any output may be NULL. */
int fl_lattice_table(int lattice, int* q, int* e, double* w);

/* Set the state: rho_molar [ncomp][N] molar densities rho~_i, u [D][N] velocity
 * (NULL = rest).  Populations become the equilibrium of eq. eqLBEMCb with the
 * given densities and velocity, the force history is zero (the paper does not
 * say how populations are initialised).  FL_EDOMAIN if a node has rho~_i <= 0,
 * rho~ b_m >= 1 or a non-finite value (state unchanged). */
int fl_set_state(fl_solver* s, const double* rho_molar, const double* u);

/* Advance nsteps time steps (synchronous: returns when the work is done).
 * FL_ENUMERIC if any step met a node outside the EOS domain. */
int fl_step(fl_solver* s, long nsteps);

/* Same, but also times each kernel of the step with HIP events on the
 * solver's stream.  kernel_ms[k] receives the summed milliseconds of kernel k
 * over the nsteps steps, names[k] (optional) a static name; *nkernels (in:
 * capacity, out: count).  The kernels are the moments pass and the collide
 * pass (2), the one-launch step (1), or with the isotropic stencils the
 * moments, collide and interface-Laplacian passes (3; FL_EINVAL for a
 * capacity below the count). */
int fl_step_timed(fl_solver* s, long nsteps, double* kernel_ms, const char** names,
                  int* nkernels);

/* Same as fl_step_timed, but with the events only around the kernels of
 * every `every`-th step (steps 0, every, 2 every, ... of this call), so that
 * a long timed run carries a small fraction of the event overhead.
 * kernel_ms[k] is summed over the timed steps; *timed_steps (optional)
 * receives their number.  FL_EINVAL for every < 1. */
int fl_step_timed_every(fl_solver* s, long nsteps, long every, double* kernel_ms, const char** names,
                        int* nkernels, long* timed_steps);

/* Number of steps done since fl_set_state. */
long fl_steps_done(const fl_solver* s);

/* Macroscopic fields of the current state, any output may be NULL:
 * rho_molar [ncomp][N]; u [D][N], the velocity of step 1 (with the stored
 * force of the last step); p [N] EOS pressure (eqPREOS etc., no interface
 * term); lnf [ncomp][N]. */
int fl_get_fields(fl_solver* s, double* rho_molar, double* u, double* p, double* lnf);

/* Populations g[ncomp][Q][N] in FP64 (directions in fl_lattice_table order). */
int fl_get_populations(fl_solver* s, double* g);

/* Total mass of each component, sum over nodes and directions, FP64
 * deterministic reduction.  mass [ncomp]. */
int fl_mass(fl_solver* s, double* mass);

/* Run until the relative change rate of the densities falls below tol:
 * r = max_i max_x |rho_i(n) - rho_i(n-K)| / (K max_x rho_i(n)), checked every
 * K = check_every steps (FP64 reductions), at most max_steps.  Returns FL_OK
 * when converged, FL_ENOTCONV when max_steps was reached.  steps_done and
 * residual (may be NULL) receive the steps run and the last r. */
int fl_run_until(fl_solver* s, double tol, long check_every, long max_steps, long* steps_done,
                 double* residual);

/* Checkpoint: raw state (populations, force history, rest-population
 * reference, step count) as an opaque byte blob of fl_state_bytes bytes.
 * fl_set_state_raw restores it into a solver created with the same params. */
int fl_state_bytes(const fl_solver* s, size_t* bytes);
int fl_get_state_raw(fl_solver* s, void* host_buf, size_t bytes);
int fl_set_state_raw(fl_solver* s, const void* host_buf, size_t bytes);


/* ------------------------------------------------------------------------
 * Batched server: many independent lattices (requests) with the same
 * components, temperature and numerics, each advanced by the same update.
 * Continuous batching at the granularity of a tick: fl_server_tick advances
 * every admitted, unfinished request in ONE batched kernel launch (one
 * workgroup per request, up to `steps` steps each, each request checking its
 * own residual every check_every of its own steps, as in fl_run_until).
 * Requests are admitted and retired between ticks, as slots and pool memory
 * free up.  A request's arithmetic depends only on its own state and step
 * count, so its result is the same alone and in any mix.
 * ------------------------------------------------------------------------ */
typedef struct fl_server fl_server;

/* base: components, kij, T, R, eos, lattice, collision, tau, mrt_rates,
 * precision, force_time_level (nx, ny, nz are ignored: they come with each
 * request).  pool_bytes: device memory reserved for request state; admission
 * fails with FL_EAGAIN when a request does not fit.  max_slots: most requests
 * in flight.  hip_stream: stream for all server work (NULL: own stream). */
int fl_server_create(const fl_params* base, size_t pool_bytes, int max_slots, void* hip_stream,
                     fl_server** out);
void fl_server_destroy(fl_server* srv);
const char* fl_server_last_error(const fl_server* srv);

/* Launch tuning of the server kernel, as fl_set_tuning: keys serve (threads
 * per request workgroup: 256, 512, 1024), serve_cap (most workgroups
 * advanced per tick, oldest request first; -1 = as many as the device holds
 * at once, 0 = all running requests, one workgroup each) and serve_group
 * (a request of N nodes runs on min(N / serve_group, 8) workgroups of one
 * XCD that meet at a barrier twice per step; default 3584, 0 = one workgroup
 * per request).  Results do not depend on any of them.  FL_EINVAL
 * (unchanged) for an unknown key or value. */
int fl_server_set_tuning(fl_server* srv, const char* spec);

/* Pool bytes one request of nx*ny*nz nodes occupies. */
int fl_server_request_bytes(const fl_server* srv, int nx, int ny, int nz, size_t* bytes);

/* Admit a request: molar densities rho_molar [ncomp][nx*ny*nz] (host), run
 * until the residual of fl_run_until is below tol (checked every check_every
 * steps) or max_steps.  *id receives the request id.  FL_EAGAIN when no slot
 * or pool memory is free now, FL_EDOMAIN for an invalid initial state,
 * FL_EINVAL for bad sizes. */
int fl_server_submit(fl_server* srv, int nx, int ny, int nz, const double* rho_molar, double tol,
                     long check_every, long max_steps, uint64_t* id);

/* One tick (synchronous): the running requests, oldest first and at most as
 * many as the device holds server workgroups at once (the rest wait, admitted,
 * for a later tick), advance by up to `steps` steps each, and stop early once
 * max_ms milliseconds of device time have passed since their workgroup
 * started (checked every 8 steps, so a request may run up to 8 steps past the
 * limit; max_ms <= 0: no time limit), so that large and small requests leave
 * the tick together.  *active receives the requests still running. */
int fl_server_tick(fl_server* srv, long steps, double max_ms, int* active);

/* Ids of finished, not yet collected requests (up to cap); *n the count. */
int fl_server_poll(fl_server* srv, uint64_t* ids, int cap, int* n);

/* Collect a finished request.  Outputs (each may be NULL): rho_molar
 * [ncomp][N] molar densities (step 2), u [D][N] velocity (step 1, with the
 * request's stored force of its last step), p [N] EOS pressure (step 4, no
 * interface term), steps run, last residual, status (FL_OK converged,
 * FL_ENOTCONV max_steps reached, FL_ENUMERIC left the EOS domain) and
 * latency_s, the host-clock seconds from the request's admission
 * (fl_server_submit) to the end of the fl_server_tick that saw it finish.
 * Frees its slot and memory.  FL_EAGAIN if the request is still running,
 * FL_EINVAL for an unknown id. */
int fl_server_result(fl_server* srv, uint64_t id, double* rho_molar, double* u, double* p, long* steps,
                     double* residual, int* status, double* latency_s);

/* fl_server_result for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same outputs, computed by the same kernel, but the velocity and pressure
 * are staged in a static device array of 2^18 doubles (2 MiB), which every GPU
 * the library runs on holds until the process ends, instead of in memory
 * allocated per call.  Makes no hipMalloc, hipFree or other allocating call.
 * A request needing more than 2^18 doubles of staging, (D + 1) * N, i.e. more
 * than 87 381 D2Q9 or 65 536 D3Q19 nodes, is refused with FL_EINVAL and stays
 * collectable with fl_server_result.  Calls on one GPU share the array:
 * calls that overlap in time (servers on different streams or host threads)
 * race, and the caller must serialise them.  No element needs to start at
 * zero: a call writes every element it reads. */
int fl_server_result_noalloc(fl_server* srv, uint64_t id, double* rho_molar, double* u, double* p,
                             long* steps, double* residual, int* status, double* latency_s);

/* Occupancy: requests in flight, free slots, pool bytes in use and total. */
int fl_server_info(const fl_server* srv, int* active, int* free_slots, size_t* pool_used,
                   size_t* pool_total);

#ifdef __cplusplus
}
#endif

#endif /* FUGLBM_H */
