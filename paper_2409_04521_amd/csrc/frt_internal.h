// Internal layouts shared by the HIP kernels and the host engine of the
// ray-tracing library.  Not part of the public C ABI (include/frt.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#define FRT_MAX_BINS_I 8
#define FRT_MAX_SOLVES_PER_LAUNCH 1024

// Error bits raised on the device and surfaced by the next sync.
enum : uint32_t {
    FRT_DEVERR_QUEUE_OVERFLOW = 1u << 0,
    FRT_DEVERR_NONFINITE = 1u << 1,
};

// Cumulative photon ledger of one solve (device resident).  Photon totals are
// FP64; `in_flight_acc` collects the packets that end the current step in
// flight and becomes `in_flight` when the step closes.
struct FrtLedgerDev {
    double emitted, absorbed_HI, absorbed_sub, escaped, dropped, in_flight, in_flight_acc, lost;
    unsigned long long crossings, ray_visits, splits, n_escaped, n_dropped, n_in_flight, n_lost, rays_emitted;
    unsigned long long step_crossings, step_visits;
    unsigned int err_flags, max_items;
};

// Structure-of-arrays ray queue.  One entry is either one packet (carried
// packets and new casting) or, in a split queue, one parent whose four
// children are expanded by four consecutive lanes of the next round.
// Real-typed arrays hold float (FP32 march) or double (FP64 march).
struct FrtQueue {
    uint32_t* src;     // source index within the solve
    uint32_t* estep;   // step in which the packet's root was cast (rotation lookup)
    uint32_t* lp;      // level << 28 | NESTED pixel
    void* r;           // distance travelled from the source, cells
    void* rstop;       // distance at which this step's travel budget ends, cells
    void* w0;          // photons-per-ray scale: N0_nu = w0 * spec[src][nu] (x R_ref)
    void* tau;         // [n_bins][cap] optical depth travelled, per bin
    void* comp;        // [n_bins][cap] Kahan compensation of tau (FP32 march)
    uint32_t cap;
};

// Queue slots: carried/casting queues alternate by step parity, split queues
// alternate by round parity.
enum { FRT_QF0 = 0, FRT_QF1 = 1, FRT_QS0 = 2, FRT_QS1 = 3, FRT_NQ = 4 };

// Device descriptor of one solve.  Static fields are set at load time; the
// per-step block is rewritten before each step.
struct FrtSolveDesc {
    // grid
    int nx, ny, nz, n_bins;
    int base_level, max_level, n_src, fp64;
    double dx_cm, sigma0, R_ref;
    double r_split0;         // split radius of level 0 in cells: sqrt(3/(pi N_min))
    double r_cap;            // distance cap in cells (+inf = none)
    float floor;             // flux floor (0 = off)
    float sig_rel[FRT_MAX_BINS_I];  // sigma_nu / sigma_0
    double alpha_B, coll_ion;
    // per-step block
    uint32_t step;           // index of the step being computed
    uint32_t cur;            // carried/casting queue of this step (0/1)
    double budget;           // packet travel per step in cells (+inf = unbounded)
    float K[FRT_MAX_BINS_I]; // deposit constants R_ref sigma_nu / (dx^2 dt)
    double Kd[FRT_MAX_BINS_I];
    double dt;
    double w0_cast;          // dt / (12 * 4^L0), seconds per cast ray
    // buffers
    const void* op;          // per cell {n_HI sigma_0 dx, kappa dx}: float2 or double2
    void* op_w;              // the same buffer, writable by the chemistry kernel
    void* gamma[2];          // deposit accumulators (float or double), alternating by step
    double* x;               // neutral fraction
    const double* nH;        // hydrogen density, cm^-3
    const double* src_pos;   // n_src * 3, cells
    const float* spec;       // n_src * n_bins photon rates / R_ref (FP32 march)
    const double* specd;     // same in FP64
    double* quat;            // [quat_steps][n_src][4] (w, x, y, z) per casting step
    uint32_t quat_steps;
    const double* user_u;    // optional table of uniforms [user_steps][n_src][3]
    uint32_t user_steps;
    unsigned long long seed;
    FrtQueue q[FRT_NQ];
    uint32_t* count;         // [FRT_NQ] entry counts
    FrtLedgerDev* L;
};

// Per-launch plan for one round over several solves: prefix of work items.
struct FrtRoundPlan {
    int n_solves;
    int in_slot;             // queue slot read by this round (-1 = carried/casting of each solve)
    int out_slot;            // split queue written by this round
    int expand;              // 1: entries are parents expanded x4
    uint32_t prefix[FRT_MAX_SOLVES_PER_LAUNCH + 1];
};

// Launch wrappers (frt_kernels.hip).
namespace frt {
hipError_t launch_emit(FrtSolveDesc* d_descs, const uint32_t* d_emit_prefix, int n_solves,
                       uint32_t total_items, int fp64, hipStream_t s);
hipError_t launch_round(FrtSolveDesc* d_descs, FrtRoundPlan* d_plan, int n_solves, int round,
                        int fp64, hipStream_t s);
hipError_t launch_round_march(FrtSolveDesc* d_descs, FrtRoundPlan* d_plan, int round, int nb, int fp64,
                              hipStream_t s);
hipError_t launch_chem(FrtSolveDesc* d_descs, const unsigned long long* d_cell_prefix, int n_solves,
                       unsigned long long total_cells, int fp64, hipStream_t s);
hipError_t launch_step_end(FrtSolveDesc* d_descs, int n_solves, hipStream_t s);
hipError_t launch_prep_opacity(FrtSolveDesc* d_desc, unsigned long long ncell, int fp64, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s);
int device_sm_count();
}  // namespace frt
