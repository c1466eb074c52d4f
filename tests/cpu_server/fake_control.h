// Controls of the CPU stand-in backend (fake_backend.cpp) for the serving
// layer's tests: injected failures, counters, the virtual clock.
#pragma once
#include <cstdint>

namespace fake {

struct Faults {
    int create_fail_at = 0;         // the k-th frt_solve_create (from 1) fails with FRT_ENOMEM; 0: none
    int load_fail_at = 0;           // the k-th frt_load_grid fails with FRT_ENOMEM; 0: none
    double step_fail_tag = -1.0;    // a batched step holding the solve of this tag while it
    int64_t step_fail_step = -1;    // stands at this step fails with this code (also when the
    int step_fail_code = 0;         // solve is stepped alone); 0: none
    int pass_growth = 1;            // a batch's pass queues need this many times the first
                                    // size the solves asked for (queues that grew)
};

// Install the failures and zero the call counters (not the live count).
void reset(const Faults& f);
// While held, grid uploads wait at their start, and batched steps at
// theirs (so that requests can be lined up before any of them steps);
// loads_started() and loads_done() count the uploads that began and that
// ended since reset.
void hold_loads(bool hold);
void hold_steps(bool hold);
int loads_started();
int loads_done();
int live_solves();                  // created and not yet destroyed
uint64_t batches();                 // batched steps applied since reset
uint64_t max_batch();               // most solves in one applied batched step
void advance_clock(double seconds); // virtual time passing outside the library (arrivals)
double expected_x(double tag, uint64_t steps, uint64_t cell);
double expected_T(double tag, uint64_t steps, uint64_t cell);   // with the temperature on
uint64_t cell_bytes();              // resident bytes per cell of a solve
uint64_t pass_bytes_per_cell();     // pass-queue bytes per cell a solve asks for

}  // namespace fake
