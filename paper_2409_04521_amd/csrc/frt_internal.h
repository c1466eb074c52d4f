// Internal layouts shared by the HIP kernels and the host engine of the
// ray-tracing library.  Not part of the public C ABI (include/frt.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "frt.h"
#include "frt_serving.h"

#define FRT_MAX_BINS_I 8

// Bricks of the LDS-staged march, edges 2^l per axis (x, y, z).  The FP32
// march without sub-grid opacity stages 32 x 16 x 16 cells (32 KiB of HI
// opacity, 64 KiB of 64-bit fixed-point deposits) for one 1024-thread
// workgroup per CU; with sub-grid opacity 16^3 cells (both opacity parts and
// the fixed-point deposits, 64 KiB) for 256-thread workgroups; the FP64
// march 8^3.
constexpr int FRT_BRICK_LOG_BIG[3] = {5, 4, 4};
constexpr int FRT_BRICK_LOG_SUB[3] = {4, 4, 4};
constexpr int FRT_BRICK_LOG_F64[3] = {3, 3, 3};
// Packets handed to a 256-thread march workgroup per work item, at most (the
// launch's item size is a tunable); the 1024-thread workgroup takes
// FRT_BIG_ITEM_SCALE times as many.
constexpr uint32_t FRT_ITEM_RAYS = 1024;
constexpr uint32_t FRT_BIG_ITEM_SCALE = 8;
constexpr uint32_t FRT_ITEM_MAX = FRT_BIG_ITEM_SCALE * FRT_ITEM_RAYS;
// March scratch records per CU: room for the split children a workgroup keeps
// in its brick, twice the largest work item (more go to the next pass).
constexpr uint32_t FRT_XREC_PER_CU = 2 * FRT_ITEM_MAX;
// Ledger accumulators are striped to keep atomics off a single address.
constexpr int FRT_STRIPES = 64;
// The pass output buffers are cut into FRT_QSEG equal segments,
// each with its own fill counter (FRT_QSEG_STRIDE words apart, one cache
// line each); workgroup b appends to segment b % FRT_QSEG, so appends from
// different workgroups seldom meet on one counter.
constexpr int FRT_QSEG = 64;
// Pass-output keys: brick key in the low FRT_KEY_BITS bits, the packet's
// expected crossings in the next brick (0 .. FRT_KEY_BINS - 1) above them.
constexpr int FRT_KEY_BITS = 26;
constexpr uint32_t FRT_KEY_MASK = (1u << FRT_KEY_BITS) - 1u;
// Key of an output slot that holds no packet (a split child that escaped).
constexpr uint32_t FRT_KEY_NONE = 0xffffffffu;
constexpr int FRT_KEY_BINS = 64;
constexpr int FRT_QSEG_STRIDE = 32;

// Error bits raised on the device and surfaced by the next sync.
enum : uint32_t {
    FRT_DEVERR_QUEUE_OVERFLOW = 1u << 0,   // a pass queue (O, P, S, work list) was too small
    FRT_DEVERR_UNFINISHED = 1u << 1,       // packets left after the last pass (never expected)
    FRT_DEVERR_CARRY_OVERFLOW = 1u << 2,   // a solve's carried-packet queue was too small
};

// Photon terms (double) and counters (u64) accumulated during a step.
// (In the Generalized Opacity Mode, which has no sub-grid term, the
// LF_ABS_SUB stripe carries the photons stopped at I-fronts.)
enum { LF_EMITTED, LF_ABS_HI, LF_ABS_SUB, LF_ESC, LF_DROP, LF_FLIGHT, LF_LOST, LF_HEAT, LF_NF };
enum { LC_CROSS, LC_VISITS, LC_SPLITS, LC_NESC, LC_NDROP, LC_NFLIGHT, LC_EMITTED, LC_NC };

// Cumulative photon ledger of one solve (device resident).  During a step
// the kernels add into the stripes; the step-end kernel folds them in.
struct FrtLedgerDev {
    double emitted, absorbed_HI, absorbed_sub, escaped, dropped, in_flight, lost, absorbed_front;
    unsigned long long crossings, ray_visits, splits, n_escaped, n_dropped, n_in_flight, rays_emitted;
    unsigned long long step_crossings;
    unsigned int err_flags, max_items;
    double merge_residual;                      // photons before minus after the merges (rounding)
    unsigned long long merges, rays_merged;     // merged packets made, packets merged into them
    double front_excess;                        // front photons beyond the atoms their cells had left
    double heat_in;                             // photo-heating given to the gas, eV (temperature on)
    double sd[FRT_STRIPES][LF_NF];
    unsigned long long sc[FRT_STRIPES][LC_NC];
};

// Packet records, one 16-byte-aligned struct per packet (64 bytes in FP32,
// 112 in FP64), so that a packet is read or written with four (seven)
// 16-byte accesses wherever it sits.  A packet is always at src + r * dir
// (children are re-centred on their own pixel directions at the split
// radius), and `cell` is the cell it is in, so a visit resumes exactly where
// the last one stopped.
template <typename Real>
struct alignas(16) FrtRec {
    uint32_t src;      // source index within the solve
    uint32_t estep;    // step in which the packet's root was cast (rotation lookup)
    uint32_t lp;       // level << 28 | NESTED pixel
    uint32_t cell;     // cell coordinates x | y << 11 | z << 22
    uint32_t key;      // pass outputs: global brick key and crossing bin (FRT_KEY_BITS);
                       // sorted packets: the crossing bin; carried packets: solve-local key
    Real r;            // distance travelled from the source, cells
    Real rstop;        // distance at which this step's travel budget ends, cells
    Real w0;           // photons scale: N0_nu = w0 * spec[src][nu] (times R_ref)
    Real dir[3];       // unit direction (rotated pixel centre)
    Real tau[4];       // optical depth travelled: HI part at sigma_0 (A), sub-grid
                       // part (K), and their Kahan compensations; bin nu has
                       // tau_nu = (sigma_nu / sigma_0) A + K
};
static_assert(sizeof(FrtRec<float>) == 64, "FP32 packet record is 64 bytes");
static_assert(sizeof(FrtRec<double>) == 112, "FP64 packet record is 112 bytes");
static_assert(offsetof(FrtRec<float>, key) == 16 && offsetof(FrtRec<double>, key) == 16,
              "the key is the first word of a record's second 16 bytes");

// Virtual origin of a packet made by merging (§3.3): the point it travels
// from, the rotation of its HEALPix pixels and its photons per bin relative
// to R_ref w0 (at most 1).  Packets refer to an entry through their source
// index with FRT_VSRC set.
struct alignas(16) FrtVSrc {
    double pos[3];              // cells
    double q[4];                // (w, x, y, z)
    double spec[FRT_MAX_BINS_I];
};
constexpr uint32_t FRT_VSRC = 0x80000000u;

// A queue of packet records (FrtRec<float> or FrtRec<double>).
struct FrtRecs {
    void* rec;
    uint32_t cap;
};

// Device descriptor of one solve.  Static fields are set at load time; the
// per-step block is rewritten before each step; key_base depends on the
// launch the solve is part of.
struct FrtSolveDesc {
    int nx, ny, nz, n_bins;
    int base_level, max_level, n_src, fp64;
    int has_sub;                // some cell has kappa > 0 (always, in the Generalized Opacity Mode)
    int bpx, bpy, bpz;          // bricks per axis
    int bsh[3];                 // log2 of the brick edge per axis
    uint32_t key_base;          // first global brick key of this solve in the launch
    uint32_t ncast;             // 12 * 4^L0
    double dx_cm, sigma0, R_ref;
    double r_split0;            // split radius of level 0 in cells: sqrt(3/(pi N_min))
    double r_cap;               // distance cap in cells (+inf = none)
    float floor;                // flux floor (0 = off)
    float sig_rel[FRT_MAX_BINS_I];
    double sig_reld[FRT_MAX_BINS_I];  // sigma_nu / sigma_0 for the FP64 march
    float sig_l2[FRT_MAX_BINS_I];    // -log2(e) sig_rel: e^-(sig_rel t) = 2^(sig_l2 t)
    double alpha_B, coll_ion;
    // per-step block
    uint32_t step;              // index of the step being computed
    uint32_t cur;               // carried queue read this step (0/1)
    double budget;              // packet travel per step in cells (+inf = unbounded)
    float K[FRT_MAX_BINS_I];    // deposit constants R_ref sigma_nu / (dx^2 dt)
    double Kd[FRT_MAX_BINS_I];
    float KS;                   // K_nu / (sigma_nu / sigma_0), the same for every bin
    double KSd;
    double dt;
    double w0_cast;             // dt / (12 * 4^L0), seconds per cast packet
    float dep_scale;            // fixed-point deposit units per unit deposit: 2^46 over the largest
                                // deposit of one crossing (the photons of the brightest packet the
                                // solve can hold, n_bins times the largest w0; with sub-grid
                                // opacity times 2 max K_nu)
    // buffers
    const void* op_a;           // per cell n_HI sigma_0 dx (float or double)
    const void* op_b;           // per cell kappa dx (float or double)
    void* op_aw;                // op_a, written by the chemistry
    void* gamma[2];             // deposit accumulators, alternating by step
    double* x;                  // neutral fraction
    const double* nH;           // hydrogen density, cm^-3
    const double* src_pos;      // n_src * 3, cells
    const float* spec;          // n_src * n_bins photon rates / R_ref
    const double* specd;
    double* quat;               // [quat_steps][n_src][4] (w, x, y, z) per casting step
    uint32_t quat_steps;
    const double* user_u;       // optional uniforms [user_steps][n_src][3]
    uint32_t user_steps;
    unsigned long long seed;
    FrtRecs F[2];               // carried packets, alternating by step
    uint32_t* fcount;           // [2]
    FrtLedgerDev* L;
    // time-averaged chemistry: the latest <x> of every cell, and the ledger
    // and carried-queue counters of the start of the step, which every march
    // of the step starts from
    double* xavg;               // [ncell], or null with backward-Euler chemistry
    FrtLedgerDev* L_snap;
    uint32_t* fcount_snap;
    // Generalized Opacity Mode: op_b holds each cell's ionized fraction
    int gen;
    double front_atoms;         // (1 + chi) V: times n_H, the atoms a front photon ionizes
    void* op_bw;                // op_b, written by this mode's chemistry
    double* front;              // [ncell] photons stopped at each cell's front this step (or null)
    // ray merging (§3.3): virtual origins of merged packets in two tables used
    // in turn like the carried queues (the packets carried into step k, and
    // their children, refer to table k & 1); vcount [2] their entries
    int merge;
    FrtVSrc* vt[2];
    uint32_t* vcount;
    double dep_base;            // dep_scale times the largest w0 held (merging solves)
    double w0_hi;               // largest w0 of a cast packet so far
    float* w0_merged;           // largest w0 of a merged packet (device, merging solves)
    // Generalized Opacity Mode with K >= 1 marches per step: the input kappa
    // dx (march precision), from which each march's ionized-gas opacity is
    // rebuilt with the equilibrium n_HI of the last rate
    const void* kin;
    // temperature evolution (§4.1, Eq. temp_evolution_standard): T of every
    // cell, this step's photo-heating rate of every cell (march precision;
    // cleared by the chemistry) and the energy above 13.6 eV left per photon
    // of each bin that HI absorbs
    int temp;
    double* T;                  // [ncell] K, or null
    void* heat;                 // [ncell] photo-heating rate of the step, erg/cm^3/s, or null
    double heat_scale;          // erg/cm^3/s per eV left in a cell during the step
    double heat_ev[FRT_MAX_BINS_I];
    double hubble;              // H(z) of the adiabatic term, 1/s
    double cmb_z;               // CMB redshift of Compton cooling (< 0: none)
    // Generalized Opacity Mode: temperature of gas the front ionizes (K) and
    // the photo-heating per case-A recombination of the ionized gas (erg)
    double t_reion;
    double heat_rec;
};

// One work item of a pass: up to FRT_ITEM_RAYS packets of one brick.
struct FrtWork {
    uint32_t key, start, count, solve;
};

// Launch counters.  C_HALT and C_DONE serve steps replayed from a HIP graph
// several times between host reads: the end of a replayed step that raised
// an error sets C_HALT, after which every kernel of the later replays returns
// at once (the failed step's start stays as the step left it, for the
// restore); C_DONE counts the replayed steps that were applied.  Both are
// reset only by a CLEAR_ALL.
enum { C_NOS = 0, C_NP, C_NWORK, C_ERR, C_MAXP, C_NEXT, C_HALT, C_DONE, C_NCTR = 8 };

// k_clear modes: the first march of a step (keeps C_HALT and C_DONE), a
// later march of the same step (also keeps the error bits and the largest
// pass), and a full reset (every counter, also under a halt).
enum { CLEAR_STEP = 0, CLEAR_ITER = 1, CLEAR_ALL = 2 };

// Per-launch workspace: unsorted pass outputs O, packets sorted by brick P,
// packets that reached their split radius S (with their photons), per-key
// histogram and scatter cursors, the work list, counters.
struct FrtWS {
    // pass outputs, double-buffered: a launch appends to buf[out] (records,
    // and each record's key in bkey[out]) and reads the previous pass's
    // outputs from buf[out ^ 1] through `sorted`
    FrtRecs buf[2];
    uint32_t* bkey[2];
    int out;
    uint2* sorted;              // [pcap] (record index in the input buffer, crossing bin) in brick order
    uint32_t pcap;
    void* xrec;                 // [xrec_cap] march scratch: split children kept in their parent's brick,
    uint32_t xrec_cap;          // an equal share per workgroup
    uint32_t* segc;             // [FRT_QSEG][FRT_QSEG_STRIDE] fill counters of the output segments
    uint32_t* segp;             // [FRT_QSEG + 1] first input entry of each segment in pass order
    uint32_t* ctr;              // [C_NCTR]
    uint32_t* hist;             // [nkeys]
    uint32_t* cursor;           // [nkeys]
    FrtWork* work;
    uint32_t cap_work;
    uint32_t nkeys;
    const uint32_t* key_prefix; // [n_solves + 1] brick-key base per solve
    uint32_t* seed_prefix;      // [n_solves + 1] seeding items per solve
    int n_solves;
    int n_bins;
    int has_sub;                // some solve of the launch has sub-grid opacity
    int has_heat;               // some solve of the launch takes photo-heating from the march
    int has_temp;               // some solve of the launch evolves its temperature
    // launch shape (tunable)
    uint32_t item_rays;         // packets per work item, 64..FRT_ITEM_RAYS
    int scatter_bpc;            // workgroups per CU of the scatter pass
};

// Scratch of the allocation-free step (frt_step_static): the pass workspace
// of one small solve in a file-scope device array of this many bytes, which
// every GPU the library runs on holds until the process ends; at most this
// many brick keys and this many march scratch records per compute unit.
constexpr size_t FRT_STATIC_SCRATCH_BYTES = size_t(48) << 20;
constexpr uint32_t FRT_STATIC_MAX_KEYS = 4096;
constexpr uint32_t FRT_STATIC_XREC_PER_CU = 256;

// Arguments of the merge launches of one solve (device buffers of the
// context's merge scratch; n carried packets, n_old entries in the table
// they refer to, E exempt packets).
struct FrtMergeArgs {
    uint32_t n, n_old;
    uint64_t E;
    int level;                  // l_merge
    int all_exempt;             // E >= n: nothing merges, entries are only renumbered
    int end_bit;                // bits of the group key the sort uses
    unsigned long long key_mask;
    void* pkey;                 // [n] photons (march precision)
    void* pkey_sorted;          // [n] the same, descending
    unsigned long long* gkey;   // [n] cell << 20 | pixel, or all ones for exempt packets
    unsigned long long* gkey_s; // [n] sorted
    uint32_t* idx;              // [n] packet index
    uint32_t* idx_s;            // [n] in group-key order
    uint32_t* flag_out;         // [n] 1: writes an output packet
    uint32_t* slot;             // [n] its output slot
    uint32_t* flag_lead;        // [n] 1: first packet of a group of two or more
    uint32_t* gid;              // [n] the group's merged-packet ordinal
    uint32_t* ref;              // [n_old] 1: an old table entry still referred to
    uint32_t* vmap;             // [n_old] its entry in the new table
    uint32_t* counts;           // [4] outputs, merged packets, kept entries
    double* residual;           // [1] photons before minus after
    unsigned long long* stats;  // [2] merged packets, packets merged into them
    void* dst;                  // [n] output records (the solve's other carried queue)
    double* acc;                // [n_slots][7 + FRT_MAX_BINS_I] sums of the groups that span waves
    uint32_t* acc_head;         // [n_slots] sorted position of such a group's first packet, or all ones
    uint32_t n_slots;           // (n + 63) / 64
    void* temp;                 // sort and scan storage
    size_t temp_bytes;
};

namespace frt {
// Merge the packets a solve carries into the next step (§3.3); d is the
// solve's descriptor of the step just run.  Phase 0 counts (a.counts:
// output packets, merged packets, kept table entries), phase 1 writes the
// next table of virtual origins, which must hold counts[1] + counts[2].
hipError_t launch_merge(FrtSolveDesc* d, const FrtMergeArgs& a, int fp64, int n_bins, int phase, hipStream_t st);
size_t merge_temp_bytes(uint32_t n, uint32_t n_old, int fp64);
// Device address of the static scratch on `device` (which must be current),
// looked up with hipGetSymbolAddress on the first call per device and kept.
hipError_t static_scratch(int device, void** ptr);
hipError_t launch_seed(FrtSolveDesc* d, const FrtWS& ws, int fp64, hipStream_t s);
// part 0: counting scan, 1: scatter into brick order, 2: brick march
// (which also writes the children of the packets that split)
hipError_t launch_pass(FrtSolveDesc* d, const FrtWS& ws, int fp64, int part, hipStream_t s);
hipError_t launch_finish(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s);
// The chemistry of every solve of a launch; `launch_err` is the launch's
// error word (device): when it is set no solve's state changes.  `temp`:
// some solve of the launch evolves its temperature (the kernels that do are
// separate, so that the others keep their occupancy).
hipError_t launch_chem(FrtSolveDesc* d, const unsigned long long* d_cell_prefix, int n_solves,
                       unsigned long long total_cells, int fp64, int temp, const uint32_t* launch_err, hipStream_t s);
hipError_t launch_prep_opacity(FrtSolveDesc* d_desc, unsigned long long ncell, int fp64, hipStream_t s);
// n_H <- nH_new (device, double) with the compression term on T (null: none);
// m0, m1 are the grid's mean density before and after.
hipError_t launch_set_density(double* nH, const double* nH_new, double* T, double m0, double m1,
                              unsigned long long ncell, hipStream_t s);
// Clear the launch counters and brick histogram (a kernel, so that a step
// captured in a HIP graph holds no memset node); mode is a CLEAR_* value.
hipError_t launch_clear(const FrtWS& ws, int mode, hipStream_t s);
// `halt` (device, may be null) is the launch's C_HALT word: when it is set
// the kernel does nothing.  Steps launched one by one pass null.
hipError_t launch_chem_avg(FrtSolveDesc* d, const unsigned long long* d_cell_prefix, int n_solves,
                           unsigned long long total_cells, int fp64, int temp, int phase, const uint32_t* launch_err,
                           const uint32_t* halt, hipStream_t s);
hipError_t launch_iter_restart(FrtSolveDesc* d, int n_solves, const uint32_t* halt, hipStream_t s);
hipError_t launch_snapshot(FrtSolveDesc* d, int n_solves, const uint32_t* halt, hipStream_t s);
// End of a step replayed from a HIP graph: advance every solve's step index
// on the device and count the step in C_DONE, or, if the step raised an
// error, set C_HALT instead.
hipError_t launch_advance(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s);
// Device-rate measurements (frt_microbench.hip): a streaming copy of
// `bytes` (variant 0: one 16-byte access per lane and iteration; 1: four in
// flight, non-temporal), and `per_lane` FP32 atomic additions per lane at
// random slots.
hipError_t microbench_copy(const void* a, void* b, size_t bytes, int variant, hipStream_t s);
hipError_t microbench_atomic(float* buf, uint32_t slots, int per_lane, int grid, uint32_t seed, hipStream_t s);
// Query launch shapes once, outside any stream capture.
void prime_launch_shapes(int fp64, int n_bins, int has_sub, int has_heat);
int device_cu_count();
}  // namespace frt
