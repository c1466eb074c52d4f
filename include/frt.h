/*
 * frt.h — C ABI of the MI355X ray-tracing library (libfrt.so).
 *
 * Adaptive ray tracing of ionizing photon packets from point sources
 * through a uniform Cartesian grid, after Cain & D'Aloisio, "FlexRT I"
 * (§3 ray casting, transport and splitting; §4.1 deposition and the
 * hydrogen ionization balance).  One step of length dt:
 *   1. every source casts 12 * 4^L0 packets on its HEALPix sphere, rotated
 *      at random each step (§3.1, Eq. Nray); packets carried from earlier
 *      steps resume;
 *   2. each packet walks cell by cell, losing exp(-tau) per cell with
 *      tau = (n_HI sigma_nu + kappa_sub) ds (§4.1, Eq. tau_cell) and
 *      depositing its absorbed photons into the cell's photo-ionization rate
 *      (Eqs. gamma_initial_standard / gamma_avg_subgrid);
 *   3. a packet splits into four children at r_split(l) (§3.2, Eqs. r_split,
 *      lhpx), and ends when it leaves the box, falls below the flux floor,
 *      reaches the distance cap, or has travelled c_ray * dt this step;
 *   4. a backward-Euler update of the neutral fraction x_HI per cell closes
 *      the step (Eq. ion_balance_eqn discretized implicitly).
 * Per solve, two further forms of §4 (frt_params): the time-averaged update
 * of §4.1 iterated over several marches of the step (chem_iterations), and
 * the Generalized Opacity Mode of §4.2 (opacity_mode), in which each cell's
 * ionized part absorbs with a given kappa and packets stop at moving-screen
 * I-fronts that the step's stopped photons advance.
 *
 * Conventions
 *   - Every function returns an int status: FRT_OK (0) or a negative
 *     FRT_E* code; frt_last_error() gives the calling thread's message for
 *     the last failure.  No exception crosses the ABI.
 *   - Grids are C order [z][y][x] (x fastest): cell (i,j,k) has index
 *     i + nx*(j + ny*k) and spans [i dx, (i+1) dx) on x, etc.  Cells are
 *     cubes of edge dx = box_cm / nx.
 *   - Units are cgs: cm, s, cm^-3, cm^2, photons.
 *   - ptr_kind FRT_HOST means host memory, FRT_DEVICE means memory of the
 *     context's HIP device.  Inputs are always copied into buffers the
 *     library owns; the caller keeps ownership of its arrays.
 *   - Work is enqueued on the solve's HIP stream (the one given at
 *     creation, else a stream the library creates).  Steps wait for their
 *     own end and report a queue overflow themselves; frt_sync reports any
 *     other device error bit left behind.
 *   - A solve handle is not thread-safe; different solves may be driven from
 *     different threads.
 */
#ifndef FRT_H
#define FRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FRT_OK 0
#define FRT_EINVAL (-1)     /* invalid argument (sizes, NaN/negative input, source outside box) */
#define FRT_ENOMEM (-2)     /* device or host allocation failed */
#define FRT_EDEVICE (-3)    /* HIP runtime error */
#define FRT_EOVERFLOW (-4)  /* ray queue exceeded queue_capacity; the step was not applied */
#define FRT_ESTATE (-5)     /* call out of order (e.g. step before grid and sources are loaded) */

#define FRT_HOST 0
#define FRT_DEVICE 1

#define FRT_F32 0           /* FP32 march, Kahan-compensated tau; FP64 chemistry and ledger */
#define FRT_F64 1           /* FP64 march (validation) */

#define FRT_MAX_BINS 8
#define FRT_MAX_CHEM_ITERATIONS 64

#define FRT_STANDARD 0      /* opacity from n_HI = n_H x_HI and the sub-grid kappa (§4.1) */
#define FRT_GENERALIZED 1   /* Generalized Opacity Mode (§4.2) */

typedef struct frt_ctx_s* frt_ctx;
typedef struct frt_solve_s* frt_solve;

/* Parameters of one solve.  Set .size = sizeof(frt_params) and start from
 * frt_params_default(). */
typedef struct {
    size_t size;
    int n_bins;                     /* frequency bins, 1..FRT_MAX_BINS */
    double sigma_bins[FRT_MAX_BINS];/* HI photo-ionization cross-section per bin, cm^2 (> 0) */
    double alpha_B;                 /* recombination coefficient at the fixed T, cm^3/s */
    double coll_ion;                /* collisional ionization coefficient, cm^3/s (default 0) */
    int base_level;                 /* HEALPix level l_hpx of cast packets (§3.1), 0..8 */
    int max_level;                  /* packets at this level never split, base_level..12 */
    double n_ray_min;               /* N_ray^min of Eq. r_split (> 0; default 1) */
    double flux_floor;              /* drop a packet when its photons fall below this fraction
                                       of its cast photons (divided by 4 per split); 0 = off */
    double max_distance_cm;         /* drop packets this far from their source; 0 = off */
    double c_ray_cm_s;              /* packet speed; +INFINITY finishes every packet within its step */
    int march_precision;            /* FRT_F32 (default) or FRT_F64 */
    uint64_t seed;                  /* stream of the per-step random sphere rotations */
    uint64_t queue_capacity;        /* entries per ray queue; 0 = sized automatically and grown
                                       (the step is re-run) when a step overflows.  A fixed
                                       capacity is cut into 64 equal segments, one per group
                                       of workgroups, and a full segment is an overflow */
    uint64_t queue_hint;            /* automatic sizing only: first size of the pass queues in
                                       entries (0 = from the grid and source counts) */
    int chem_iterations;            /* hydrogen update of a step (§4.1).  0 (default): backward
                                       Euler of Eq. ion_balance_eqn with the step's Gamma.
                                       K in 1..FRT_MAX_CHEM_ITERATIONS: the time-averaged update
                                       (Eqs. xi_of_t, xeq, ti, avg_xi) with K marches per step;
                                       march k > 1 sees n_HI = n_H <x> from march k-1 (Eq.
                                       gamma_updated_standard) and n_e = n_H (1 - <x>) of the
                                       previous estimate (first: the start of the step); only
                                       the last march's deposits, ledger terms and carried
                                       packets are kept.  In the Generalized Opacity Mode, K
                                       marches per step iterate the ionized gas's opacity with
                                       Gamma (§4.2) using photo-ionization equilibrium (§5.1,
                                       Eqs. subgrid_lambda, equilibrium_condition, subgrid_nHI):
                                       kappa = kappa_sub + sigma_0 min(n_H, alpha_B n_H^2 / Gamma)
                                       with Gamma of the march before, at a step's first march
                                       the previous step's (optically thin, n_HI = 0, where no
                                       rate is known yet); the previous step's rate field is
                                       then part of the state (checkpoints and bookmarks keep
                                       it) */
    int opacity_mode;               /* FRT_STANDARD (default) or FRT_GENERALIZED (§4.2): then
                                       kappa_sub of frt_load_grid is the absorption coefficient
                                       of each cell's ionized part at sigma_0 (kappa_nu = kappa
                                       sigma_nu / sigma_0) and 1 - x_HI its ionized volume
                                       fraction x_ion behind a moving screen: a segment crosses
                                       x_ion ds of ionized gas, depositing Eq. gamma_avg_subgrid
                                       with ds -> x_ion ds, V -> x_ion V; in a cell not fully
                                       ionized the photons left stop at the front (the packet
                                       ends, ledger term absorbed_front), and the step's front
                                       photons advance x_ion by f / ((1 + he_chi) n_H V)
                                       (Eq. dxidt), at most to 1 (photons beyond the atoms a
                                       cell had left are ledger term front_excess).  With
                                       chem_iterations K >= 1 the opacity of the ionized gas is
                                       iterated with Gamma (see chem_iterations) */
    double he_chi;                  /* chi of Eq. dxidt: helium singly ionized per hydrogen
                                       atom (default 0) */
    int merge;                      /* ray merging (§3.3), 0 (default) or 1: at the end of each
                                       step the floor(merge_exempt N_cells) brightest carried
                                       packets are exempt and the others are merged per cell
                                       and per pixel of that cell's randomly rotated HEALPix
                                       sphere of level merge_level (Eq. Nray_per_cell_max:
                                       at most merge_exempt + 12 4^merge_level packets per
                                       cell); a merged packet sums the photons of its
                                       members, travels along the pixel's centre from their
                                       photon-weighted mean position, distance and level, and
                                       splits like any packet.  Only carried packets merge
                                       (nothing with c_ray = +INFINITY) */
    int merge_level;                /* l_merge, 0..8 (default 0) */
    double merge_exempt;            /* N_ex, exempt packets per cell, >= 0 (default 4) */
    int temperature;                /* 1: the gas temperature evolves (§4.1, Eq.
                                       temp_evolution_standard, static density).  Standard Mode:
                                       each bin's photons absorbed by HI (not by the
                                       sub-grid absorbers) leave heat_ev of the bin each in the
                                       cell; the hydrogen update takes case-B recombination and
                                       collisional ionization at the cell's temperature of the
                                       start of the step (Hui & Gnedin 1997) instead of alpha_B
                                       and coll_ion; after it, T keeps n_tot T as the particle
                                       number n_tot = n_H (2 - x_HI) changes, cools by e^(-2 H dt)
                                       with hubble_s, and follows photo-heating minus recombination,
                                       collisional ionization and excitation, free-free and (with
                                       cmb_z >= 0) Compton cooling over the step, in sub-steps of at
                                       most a tenth change in T, each solved exactly for the
                                       equation linearized about its start.  With chem_iterations K
                                       only the last march's heating counts.  Generalized
                                       Opacity Mode (§4.2): T is the temperature of each cell's
                                       ionized part.  Gas that the front ionizes in a step
                                       enters at t_reion_k and mixes by volume with the older
                                       ionized gas, which cools by e^(-2 H dt) and follows
                                       photo-heating minus the same cooling over the step (in
                                       the same sub-steps) with n_HI / n_H = y = min(1,
                                       alpha_B(T) n_H / Gamma) from photo-ionization equilibrium
                                       with the step's Gamma (y = 1 where Gamma = 0), n_e =
                                       n_HII = n_H (1 - y), n_tot = n_H (2 - y), and the
                                       photo-heating of Eq. analytical_heating_HI for a power
                                       law of index spectral_index cut at 4 Ryd (case-A
                                       recombination, Hui & Gnedin 1997); heat_ev is unused and
                                       the opacity iteration takes alpha_B(T); cells with no
                                       ionized gas keep T.  A solve with the temperature on
                                       marches with 16^3 bricks in FP32.
                                       0 (default): T fixed */
    double heat_ev[FRT_MAX_BINS];   /* energy above 13.6 eV left in the gas per photon of each
                                       bin that HI absorbs, eV (finite, >= 0) */
    double hubble_s;                /* H(z) of the adiabatic term, 1/s (finite, >= 0; default 0) */
    double cmb_z;                   /* redshift of the CMB for Compton cooling; < 0: none
                                       (default -1) */
    double t_reion_k;               /* Generalized Opacity Mode with the temperature on:
                                       temperature of gas the front ionizes, K (finite, > 0;
                                       default 2e4) */
    double spectral_index;          /* Generalized Opacity Mode with the temperature on:
                                       power-law index alpha of the ionizing spectrum in the
                                       photo-heating estimate (finite, >= 0; default 1.5) */
} frt_params;

/* Cumulative photon ledger (photons) and counters of one solve.  With
 * E = emitted, the terms satisfy E = absorbed_HI + absorbed_sub + escaped
 * + dropped + in_flight + absorbed_front + front_excess + merge_residual
 * (+ lost, which is 0 unless a queue overflowed).  In the Generalized Opacity Mode absorbed_HI counts the
 * photons absorbed in ionized gas. */
typedef struct {
    double emitted, absorbed_HI, absorbed_sub, escaped, dropped, in_flight, lost;
    uint64_t crossings;             /* cell crossings with ds > 0, all steps */
    uint64_t ray_visits;            /* packet visits (one per packet per round) */
    uint64_t splits, n_escaped, n_dropped, n_in_flight, rays_emitted;
    uint64_t step_crossings;        /* crossings of the last step */
    uint64_t steps;                 /* steps applied */
    uint32_t err_flags;             /* device error bits (1 = queue overflow) */
    uint32_t max_items;             /* largest round (work items) seen */
    double absorbed_front;          /* photons stopped at I-fronts (Generalized Opacity Mode) */
    double merge_residual;          /* photons the merged packets held minus those their
                                       records hold in the march's precision (rounding) */
    uint64_t merges, rays_merged;   /* merged packets made, and packets merged into them */
    double front_excess;            /* photons stopped at I-fronts beyond the neutral atoms their
                                       cells had left; they ionize nothing (absorbed_front counts
                                       the photons that did) */
    double heat_in;                 /* photo-heating the march gave the gas, erg (temperature
                                       on, Standard Mode; 0 in the Generalized Opacity Mode) */
} frt_ledger;

/* Fill *p with defaults: 1 bin at 6.3e-18 cm^2, alpha_B = 2.59e-13,
 * coll_ion = 0, base_level 0, max_level 12, n_ray_min 1, no floor, no cap,
 * c_ray = speed of light, FRT_F32, seed 0, automatic queues, no hint,
 * backward-Euler chemistry (chem_iterations 0), FRT_STANDARD opacity, he_chi 0,
 * no merging (merge 0; merge_level 0 and merge_exempt 4 when it is on),
 * temperature 0 (heat_ev 0, hubble_s 0, cmb_z -1, t_reion_k 2e4,
 * spectral_index 1.5). */
int frt_params_default(frt_params* p);

/* Device memory hooks: alloc returns `bytes` of device memory of the
 * context's device (NULL on failure, which the calling function reports as
 * FRT_ENOMEM); free gives a block back.  They let a caller route the
 * library's device memory through its own allocator (PyTorch's caching
 * allocator, say); the library frees a block only after the work using it
 * has finished on the device.  Either may be called from any thread that
 * calls into the library, including the server's worker and loader threads. */
typedef void* (*frt_alloc_fn)(size_t bytes, void* user);
typedef void (*frt_free_fn)(void* ptr, void* user);

/* Context bound to HIP device `hip_device`: the pass queues shared by the
 * solves stepped on it, its launch shape, and its device memory hooks
 * (alloc_fn and free_fn both NULL: hipMalloc / hipFree; giving only one is
 * FRT_EINVAL).  Every device buffer of the context and of its solves comes
 * from the hooks; `user` is passed to them. */
int frt_ctx_create(int hip_device, frt_alloc_fn alloc_fn, frt_free_fn free_fn, void* user, frt_ctx* out);
int frt_ctx_destroy(frt_ctx ctx);

/* Message of the calling thread's last failing call ("" if none). */
const char* frt_last_error(void);

/* A solve: one RT problem with its grid, sources, ray queues and ledger
 * resident in HBM.  `hip_stream` is a hipStream_t to enqueue on, or NULL
 * for a stream owned by the solve. */
int frt_solve_create(frt_ctx ctx, const frt_params* params, void* hip_stream, frt_solve* out);
int frt_solve_destroy(frt_solve s);

/* Load the grid (§4.1 Standard Mode state, §4.2 sub-grid opacity):
 * nx,ny,nz in 1..2048; box_cm > 0 is the x extent (cells are cubes);
 * n_H [ncell] cm^-3 (finite, >= 0); T [ncell] K (finite, > 0; may be
 * NULL): with the temperature on, the starting temperature (NULL: 1e4 K),
 * else stored for the caller and unused; kappa_sub [ncell] 1/cm
 * (finite, >= 0; NULL = 0); x_HI0 [ncell] in [0,1] (NULL = 1).  With
 * opacity_mode FRT_GENERALIZED, kappa_sub is the absorption coefficient of
 * each cell's ionized gas at sigma_0 and x_HI0 is 1 - its ionized volume
 * fraction (NULL = 1: all neutral).
 * Resets the step counter, ledger and carried packets. */
int frt_load_grid(frt_solve s, int nx, int ny, int nz, double box_cm, const float* n_H, const float* T,
                  const float* kappa_sub, const double* x_HI0, int ptr_kind);

/* Replace the absorption-coefficient field between steps, keeping the rest
 * of the state: kappa [ncell] 1/cm (finite, >= 0), the same layout as
 * kappa_sub of frt_load_grid.  In the Generalized Opacity Mode this is the
 * ionized gas's kappa that the caller's opacity model recomputes from the
 * rates and history (§4.2, Eq. lambda_nu_general); in Standard Mode the
 * sub-grid kappa, allowed only if the grid was loaded with a kappa field
 * that has some kappa > 0 (the sub-grid march).  Takes effect at the next
 * step.  FRT_ESTATE before a grid is loaded. */
int frt_set_opacity(frt_solve s, const float* kappa, int ptr_kind);

/* Replace the hydrogen density between steps, keeping the rest of the
 * state (the density a simulation hands to the next step): n_H [ncell]
 * cm^-3 (finite, >= 0, mean > 0), the layout of frt_load_grid.  With the
 * temperature on, T takes the compression term of Eq.
 * temp_evolution_standard exactly, T (Delta_new / Delta_old)^(2/3) with
 * Delta = n_H / <n_H> over the grid (a change of the mean alone is left to
 * the Hubble term, hubble_s), in cells whose density is > 0 before and
 * after.  Standard Mode's opacity is rebuilt from the new n_H and the
 * current x_HI.  Takes effect at the next step; checkpoints, bookmarks and
 * rewinds do not hold the density (set it again after restoring).
 * FRT_ESTATE before a grid is loaded or when the loaded density's mean is
 * 0; FRT_EINVAL for a bad field (nothing changes). */
int frt_set_density(frt_solve s, const float* n_H, int ptr_kind);

/* Load n_src >= 0 point sources: pos_cm [n_src][3] (x,y,z) inside
 * [0, n*dx] per axis; ndot_bins [n_src][n_bins] photons/s per bin (finite,
 * >= 0).  Requires the grid.  Sizes the ray queues. */
int frt_load_sources(frt_solve s, int n_src, const double* pos_cm, const double* ndot_bins, int ptr_kind);

/* Optional table of rotation uniforms in [0,1): uniforms [n_steps][n_src][3]
 * for steps 0..n_steps-1 (host memory).  Steps beyond the table use the
 * library's counter-based generator: u = (splitmix64(splitmix64(seed) ^
 * (step<<32 | src<<2 | k)) >> 11) * 2^-53.  A quaternion (w,x,y,z) =
 * (sqrt(u0) cos 2pi u2, sqrt(1-u0) sin 2pi u1, sqrt(1-u0) cos 2pi u1,
 * sqrt(u0) sin 2pi u2) rotates the source's sphere (Shoemake 1992). */
int frt_set_rotations(frt_solve s, int n_steps, const double* uniforms);

/* One step of length dt_s > 0: the time step of §3.1 (packets travel
 * c_ray dt_s, i.e. one cell per step when dt = dx / c_ray as in the paper),
 * in the order of the method: casting (§3.1, Eq. Nray), the march with
 * attenuation, deposition, splitting and termination (§3.1-§3.2, §4.1 Eqs.
 * tau_cell, gamma_initial_standard, r_split, lhpx), then the hydrogen
 * update of the chosen form (Eq. ion_balance_eqn by backward Euler, or
 * Eqs. xi_of_t-gamma_updated_standard) and the ledger.  Every packet of the
 * step sees the opacity of the start of the step.  The call waits for the
 * step (it reads the queue counters back).  With automatic queues a step
 * that overflowed is re-run with larger queues; with a fixed queue_capacity
 * the call returns FRT_EOVERFLOW and the solve is left exactly at the start
 * of the step (fields, carried packets, ledger, step index), so stepping may
 * go on with other parameters.  FRT_ESTATE before grid and sources are
 * loaded. */
int frt_step(frt_solve s, double dt_s);

/* frt_step without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The pass queues live in a static device array of
 * FRT_STATIC_SCRATCH_BYTES = 48 MiB that every GPU the library runs on holds
 * until the process ends (at most 4096 bricks, and about 3.2e5 packets per
 * pass in FP32, 2e5 in FP64); the solve's own buffers are those its loading
 * calls allocated.  Results equal frt_step's up to the order of floating-
 * point additions.  A step that needs more than the array holds returns
 * FRT_EOVERFLOW and is not applied (the solve stays at the start of the
 * step); a grid of more bricks is FRT_EINVAL; a solve whose rotation table
 * (64 steps from frt_load_sources, extended by frt_step) is used up is
 * FRT_ESTATE.  Kernel timing is not recorded.  Calls in one process take the
 * array one at a time, each to its end (the call waits for its step); the
 * array keeps the last call's contents, and every call clears what it needs
 * cleared. */
int frt_step_static(frt_solve s, double dt_s);

/* One step (as frt_step) of each of n solves as one set of launches: the
 * solves' bricks share one pass queue and one march launch per pass, so a
 * batch of small boxes fills the GPU as one large box does.  The solves must
 * share a context, n_bins, march_precision and queue mode (all automatic or
 * all fixed); dt_s[i] is solve i's step.  A failed batch leaves every solve
 * at the start of the step.  Waits for the step. */
int frt_batch_step(frt_solve* solves, int n, const double* dt_s);

/* n_steps steps of each of n solves (as n_steps calls of frt_batch_step).
 * With use_graph = 0 the steps are launched one by one, each waited for.
 * With use_graph = w > 0 one step of the group is captured into a HIP graph
 * and replayed n_steps times, w replays enqueued at a time with no host wait
 * between them: the descriptors and rotation tables are prepared before the
 * capture, and the step index advances on the device.  The queue counters
 * are read back after each w replays; a replayed step that overflowed makes
 * the replays after it in the same w do nothing, so the solves stay at the
 * start of that step.  With automatic queues the step is then restored, the
 * queues grow, the step is captured again and the run goes on from it; with
 * fixed queues the call returns FRT_EOVERFLOW with the failed step not
 * applied (the steps before it are).  dt_s[i] is solve i's step for every
 * step of the run.  FRT_EINVAL for use_graph < 0. */
int frt_batch_run(frt_solve* solves, int n, const double* dt_s, int n_steps, int use_graph);

/* Launch shape of the passes, shared by the solves stepped on a context. */
typedef struct {
    size_t size;                    /* sizeof(frt_tuning) */
    int item_rays;                  /* packets per march work item (the ray tile):
                                       a multiple of 64 in 64..1024; the
                                       1024-thread march (FP32 without sub-grid
                                       opacity) takes 8 times as many */
    int scatter_blocks_per_cu;      /* workgroups per CU of the pass that sorts the
                                       queue by brick (queue chunking), 1..16 */
} frt_tuning;

/* Defaults: 1024 packets per item, 8 scatter workgroups per CU. */
int frt_tuning_default(frt_tuning* t);
int frt_ctx_set_tuning(frt_ctx ctx, const frt_tuning* t);
int frt_ctx_get_tuning(frt_ctx ctx, frt_tuning* t);

/* Autotuner: times one step of the n solves (as frt_batch_step runs it,
 * best of three runs of the same step) under each candidate launch shape
 * (item_rays 256/512/1024 x scatter 4/8 workgroups per CU), after one
 * untimed step that sizes the queues; sets the fastest on the context and
 * returns it in *best.  Every
 * solve is put back exactly as it was (fields, carried packets, ledger,
 * step index, last rate field), so the call changes no result. */
int frt_autotune(frt_solve* solves, int n, const double* dt_s, frt_tuning* best);

/* Wait for the solve's stream (work enqueued by frt_rewind, loads and
 * reads); report device error bits left in the ledger: FRT_EDEVICE if a
 * step left packets after its last pass (never expected). */
int frt_sync(frt_solve s);

/* Copy out the fields the problem statement asks for (§4.1): the neutral
 * fraction x_HI [ncell] (double; in the Generalized Opacity Mode 1 minus the
 * ionized volume fraction of §4.2) and the photo-ionization rate of the last
 * step, gamma [ncell] (float, 1/s; Eq. gamma_initial_standard, or Eq.
 * gamma_avg_subgrid with sub-grid opacity; zero before the first step).
 * Either pointer may be NULL; ptr_kind says where both point.  Synchronizes
 * and returns any error frt_sync would. */
int frt_read_fields(frt_solve s, double* x_HI, float* gamma, int ptr_kind);

/* Copy out the ledger.  Synchronizes. */
int frt_read_ledger(frt_solve s, frt_ledger* out);

/* Copy out the gas temperature T [ncell] (double, K; §4.1 Eq.
 * temp_evolution_standard) to host or device memory (ptr_kind).  FRT_ESTATE
 * when the solve holds no temperature (none loaded and the temperature off).
 * Synchronizes. */
int frt_read_temperature(frt_solve s, double* T, int ptr_kind);

/* Checkpoint: x_HI, carried packets, ledger, step index and rotation state.
 * With buf == NULL, *bytes receives the size needed. */
int frt_save_state(frt_solve s, void* buf, size_t* bytes);
int frt_load_state(frt_solve s, const void* buf, size_t bytes);

/* Device-resident bookmark of the physical state: x_HI, the carried
 * packets and the step index (with its rotation stream position).
 * frt_rewind restores it with copies on the solve's stream only (no host
 * wait), rebuilds the opacity and clears the pending deposits, so the same
 * step can be repeated.  The ledger is not rewound: it keeps counting every
 * step that ran.  Used to repeat one step from a fixed initial state. */
int frt_mark(frt_solve s);
int frt_rewind(frt_solve s);

/* Per-kernel device time, measured with HIP events on the solve's stream
 * around each launch while timing is enabled (cumulative since enabling).
 * march_ms covers every march round; chem_ms the chemistry kernel; other_ms
 * casting, round planning and step bookkeeping; merge_ms the ray merging
 * after each step of a merging solve (§3.3). */
typedef struct {
    double emit_ms, march_ms, chem_ms, other_ms;
    uint64_t march_launches, chem_launches, steps;
    double merge_ms;
} frt_timing;

int frt_set_timing(frt_solve s, int enable);
int frt_read_timing(frt_solve s, frt_timing* out);   /* synchronizes */

/* ------------------------------------------------------------- serving
 * A server admits solves as they arrive and steps every admitted solve
 * together (one batched step per tick over all solves in flight, grouped by
 * n_bins and march_precision), so that requests arriving while others run
 * join the next tick: continuous batching.  A request is admitted, in
 * arrival order, when a slot is free and its estimated device bytes
 * (frt_request_bytes) fit in what the budget has left; its grid, packets and
 * ledger then stay resident until its last step, after which its results
 * are copied to host memory and its device memory is released.  A worker
 * and a loader thread per server drive the device; submit, poll, wait and
 * take may be called from any thread. */
typedef struct frt_server_s* frt_server;

typedef struct {
    size_t size;                    /* sizeof(frt_request) */
    frt_params params;              /* as for frt_solve_create */
    int nx, ny, nz;                 /* grid, as for frt_load_grid */
    double box_cm;
    const float* n_H;               /* [ncell], required */
    const float* T;                 /* [ncell] or NULL */
    const float* kappa_sub;         /* [ncell] or NULL */
    const double* x_HI0;            /* [ncell] or NULL */
    int n_src;                      /* sources, as for frt_load_sources */
    const double* pos_cm;           /* [n_src][3] */
    const double* ndot_bins;        /* [n_src][n_bins] */
    int rotation_steps;             /* optional table of rotation uniforms, as for */
    const double* rotation_uniforms;/* frt_set_rotations (0 / NULL: the generator) */
    int n_steps;                    /* steps to run, >= 0 */
    double dt_s;                    /* step length, > 0 */
    int ptr_kind;                   /* FRT_HOST or FRT_DEVICE for every array above */
} frt_request;

#define FRT_REQ_QUEUED 0
#define FRT_REQ_RUNNING 1
#define FRT_REQ_DONE 2
#define FRT_REQ_FAILED 3

/* Device bytes a request holds while admitted: its resident fields
 * (36 bytes per cell in FP32, 52 in FP64), its carried-packet queues, its
 * sources and rotations, and its share of the pass queues at their first
 * size.  Host-side arithmetic only; the same estimate the server admits by. */
int frt_request_bytes(const frt_request* req, size_t* bytes);

/* hbm_budget_bytes: device bytes the admitted requests may hold together:
 * their own buffers plus the context's shared pass queues, which the server
 * lets grow only up to what the budget leaves (a step needing more fails with
 * FRT_ENOMEM for the solves that need it, the others step on) and gives back
 * when they block an admission while nothing runs.  The context's fixed
 * march scratch (2 x 8192 packet records per compute unit) is not counted.
 * A request larger than the budget fails at admission.  max_slots: most
 * requests in flight, 1..1024.  A loader thread uploads admitted requests,
 * each solve on a HIP stream of its own, while the worker thread steps the
 * others; the solves use ctx's pass queues, which grow as the batches need. */
int frt_server_create(frt_ctx ctx, size_t hbm_budget_bytes, int max_slots, frt_server* out);

/* Copy the request's inputs (validated as by frt_load_grid and
 * frt_load_sources) and queue it; *req_id identifies it.  Non-blocking. */
int frt_server_submit(frt_server srv, const frt_request* req, uint64_t* req_id);

/* *state = FRT_REQ_QUEUED, _RUNNING, _DONE or _FAILED. */
int frt_server_poll(frt_server srv, uint64_t req_id, int* state);

/* Wait until the request is done or failed, or timeout_s seconds passed
 * (timeout_s < 0: no limit); *state as for frt_server_poll. */
int frt_server_wait(frt_server srv, uint64_t req_id, double timeout_s, int* state);

/* Results of a finished request: x_HI [ncell] (host, may be NULL) and its
 * ledger (may be NULL); the request is then forgotten.  A failed request
 * returns its error code and message; an unfinished one FRT_ESTATE. */
int frt_server_take(frt_server srv, uint64_t req_id, double* x_HI, frt_ledger* ledger);

/* The gas temperature T [ncell] (host, double, K; §4.1 Eq.
 * temp_evolution_standard) of a finished request whose params had the
 * temperature on; call it before frt_server_take, which forgets the
 * request.  FRT_ESTATE if the request is unfinished or did not evolve its
 * temperature, FRT_EINVAL for an unknown request. */
int frt_server_read_temperature(frt_server srv, uint64_t req_id, double* T);

/* Seconds since the server's creation at which the request was submitted,
 * admitted and finished (t[2] = -1 while unfinished). */
int frt_server_times(frt_server srv, uint64_t req_id, double t[3]);

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t ticks;                 /* batched steps run */
    uint64_t solve_steps;           /* request steps run (sum over ticks of solves stepped) */
    uint32_t max_in_flight;         /* most requests admitted at once */
    uint64_t bytes_in_use, peak_bytes;
} frt_server_stats;

int frt_server_get_stats(frt_server srv, frt_server_stats* out);

/* Stop the worker (requests still queued or running are dropped) and free
 * everything the server holds. */
int frt_server_destroy(frt_server srv);

/* Achievable device rates, the denominators of the march's rooflines: HBM
 * bandwidth from a streaming copy of copy_bytes (a multiple of 16, at least
 * 1 MiB) into a second buffer, counted as bytes read plus written per
 * second (the faster of two copy kernels: one 16-byte access per lane and
 * iteration, or four in flight with non-temporal accesses); and FP32 atomic additions per second whose result is not used, at
 * random addresses among atomic_slots floats (1024..2^32-1; the march
 * deposits its rates that way), 64 per lane over 8 workgroups of 256 lanes
 * per compute unit.  Each is the best of five timed runs after an untimed
 * one.  The buffers (2 copy_bytes + 4 atomic_slots) come from the context's
 * allocator and are freed before the call returns. */
typedef struct {
    size_t size;                    /* sizeof(frt_microbench_result) */
    double copy_bytes, copy_GBps;   /* bytes of one copy; (read + written) bytes per s / 1e9 */
    double atomic_ops, atomic_per_s, atomic_slots;
} frt_microbench_result;

int frt_microbench(frt_ctx ctx, size_t copy_bytes, size_t atomic_slots, frt_microbench_result* out);

/* One ray through the solve's current opacity, for checking the march
 * against exact transmission (§4.1 Eq. tau_cell: a segment ds of cell i
 * passes exp(-(n_HI sigma_nu + kappa) ds) of its photons) and the deposits
 * of Eq. gamma_initial_standard / gamma_avg_subgrid.  The packet starts at
 * o_cm (cm, inside the box) on the unit direction d (normalized here) with
 * N_bins[n_bins] photons (>= 0), and is marched by the same kernels as a
 * step (seeding, brick passes, ledger) at level 12, so it never splits; it
 * has no flux floor, distance cap or travel budget and ends when it leaves
 * the box.  Outputs: gamma_out [ncell] (float, 1/s, may be NULL; ptr_kind
 * says where it points) the rate it deposits for a step of dt_s seconds,
 * *absorbed and *escaped its photons absorbed in the box and leaving it,
 * *crossings the cells it crossed with ds > 0.  The solve's state (fields,
 * packets, ledger, step) is not changed.  FRT_ESTATE before a grid is
 * loaded; FRT_EINVAL for an origin outside the box or a zero direction. */
int frt_debug_cast(frt_solve s, const double o_cm[3], const double d[3], const double* N_bins, double dt_s,
                   float* gamma_out, int ptr_kind, double* absorbed, double* escaped, uint64_t* crossings);

/* Uniforms of a cell's merging sphere at the end of `step` (§3.3), as the
 * library draws them: u = (splitmix64(key ^ (step<<34 | cell<<2 | k)) >> 11)
 * * 2^-53, key = splitmix64(splitmix64(seed) ^ 0x6D65726765), rotation by
 * Shoemake's quaternion as for the sources. */
int frt_merge_uniforms(uint64_t seed, uint32_t step, uint32_t cell, double out[3]);

/* Rotation uniforms the library would use for (step, src) — the same
 * counter-based generator the device runs — for checking a table against. */
int frt_rotation_uniforms(uint64_t seed, uint32_t step, uint32_t src, double out[3]);

#ifdef __cplusplus
}
#endif
#endif /* FRT_H */
