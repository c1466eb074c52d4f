// Scenarios of the serving layer (frt_server.cpp) on the CPU stand-in
// backend: arrival order and slots, the memory budget, failures injected in
// a solve's creation, its upload and its steps (only that request fails, the
// others get exactly their own steps), a device failure of a whole batch,
// batches split by queue mode and n_bins, concurrent clients, destroying a
// server with requests in flight, and the request times.  Built by the CPU
// tests plain and under ThreadSanitizer and AddressSanitizer + UBSan.
// Prints one line per scenario; the exit status is the number of failed
// checks (0: all passed).
#include "fake_control.h"

#include "frt.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

namespace {

int g_failures = 0;

#define CHECK(cond)                                                                        \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            g_failures++;                                                                  \
        }                                                                                  \
    } while (0)

// A request's inputs (kept alive until it is submitted) and what it should give.
struct Input {
    std::vector<float> nH;
    std::vector<double> pos, ndot;
    frt_request r{};
    double tag = 0.0;
    int steps = 0;
    size_t ncell = 0;
};

std::unique_ptr<Input> make(double tag, int n, int steps, int n_bins = 1, uint64_t qcap = 0, int n_src = 4)
{
    std::unique_ptr<Input> in(new Input());
    in->tag = tag;
    in->steps = steps;
    in->ncell = (size_t)n * n * n;
    in->nH.assign(in->ncell, 1e-3f);
    in->nH[0] = (float)tag;
    in->pos.assign((size_t)n_src * 3, 0.5);
    in->ndot.assign((size_t)n_src * n_bins, 1e50);
    frt_request& r = in->r;
    r.size = sizeof(frt_request);
    frt_params_default(&r.params);
    r.params.n_bins = n_bins;
    for (int b = 0; b < n_bins; b++) r.params.sigma_bins[b] = 6.3e-18;
    r.params.queue_capacity = qcap;
    r.nx = r.ny = r.nz = n;
    r.box_cm = n * 1e21;
    r.n_H = in->nH.data();
    r.n_src = n_src;
    r.pos_cm = in->pos.data();
    r.ndot_bins = in->ndot.data();
    r.n_steps = steps;
    r.dt_s = 3e13;
    r.ptr_kind = FRT_HOST;
    return in;
}

size_t bytes_of(const Input& in)
{
    size_t b = 0;
    frt_request_bytes(&in.r, &b);
    return b;
}

uint64_t submit(frt_server srv, const Input& in)
{
    uint64_t id = 0;
    const int rc = frt_server_submit(srv, &in.r, &id);
    CHECK(rc == FRT_OK);
    return id;
}

int wait_state(frt_server srv, uint64_t id)
{
    int st = -1;
    CHECK(frt_server_wait(srv, id, 60.0, &st) == FRT_OK);
    return st;
}

// A finished request: exactly its own steps, its own values.
void check_done(frt_server srv, uint64_t id, const Input& in)
{
    CHECK(wait_state(srv, id) == FRT_REQ_DONE);
    std::vector<double> x(in.ncell);
    frt_ledger led{};
    const int rc = frt_server_take(srv, id, x.data(), &led);
    CHECK(rc == FRT_OK);
    if (rc != FRT_OK) return;
    CHECK(led.steps == (uint64_t)in.steps);
    const size_t probe[3] = {0, in.ncell / 2, in.ncell - 1};
    for (size_t k : probe) CHECK(x[k] == fake::expected_x(in.tag, (uint64_t)in.steps, k));
}

void check_failed(frt_server srv, uint64_t id, int code)
{
    CHECK(wait_state(srv, id) == FRT_REQ_FAILED);
    CHECK(frt_server_take(srv, id, nullptr, nullptr) == code);
    // a failed request is forgotten once taken
    CHECK(frt_server_take(srv, id, nullptr, nullptr) == FRT_EINVAL);
}

// Wait (real time, bounded) until n uploads have begun and n requests are
// admitted; an idle server admits arrivals while earlier uploads run.
void wait_admitted(frt_server srv, const std::vector<uint64_t>& id, int n_loads)
{
    auto admitted = [&] {
        for (uint64_t i : id) {
            int st = -1;
            if (frt_server_poll(srv, i, &st) != FRT_OK || st == FRT_REQ_QUEUED) return false;
        }
        return fake::loads_started() >= n_loads;
    };
    for (int k = 0; k < 20000 && !admitted(); k++) std::this_thread::sleep_for(std::chrono::microseconds(500));
    CHECK(admitted());
}

frt_server_stats stats(frt_server srv)
{
    frt_server_stats s{};
    CHECK(frt_server_get_stats(srv, &s) == FRT_OK);
    return s;
}

struct Setup {
    frt_ctx ctx = nullptr;
    frt_server srv = nullptr;
    Setup(size_t budget, int slots, const fake::Faults& f = fake::Faults())
    {
        fake::reset(f);
        CHECK(frt_ctx_create(0, nullptr, nullptr, nullptr, &ctx) == FRT_OK);
        CHECK(frt_server_create(ctx, budget, slots, &srv) == FRT_OK);
    }
    ~Setup()
    {
        frt_server_destroy(srv);
        frt_ctx_destroy(ctx);
        CHECK(fake::live_solves() == 0);
    }
};

void end(const char* name, int before)
{
    std::printf("%s %s\n", g_failures == before ? "ok" : "FAILED", name);
    std::fflush(stdout);
}

// One slot: requests run one at a time in arrival order, each admitted
// only after the previous one finished.
void one_slot_is_fifo()
{
    const int f0 = g_failures;
    {
        Setup s(size_t(1) << 40, 1);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        const int sizes[6] = {8, 16, 12, 8, 20, 10};
        for (int k = 0; k < 6; k++) in.push_back(make(k + 1, sizes[k], 3 + k));
        for (auto& i : in) id.push_back(submit(s.srv, *i));
        std::vector<double> t0, t1, t2;
        for (size_t k = 0; k < id.size(); k++) {
            CHECK(wait_state(s.srv, id[k]) == FRT_REQ_DONE);
            double t[3];
            CHECK(frt_server_times(s.srv, id[k], t) == FRT_OK);
            t0.push_back(t[0]);
            t1.push_back(t[1]);
            t2.push_back(t[2]);
        }
        for (size_t k = 0; k < id.size(); k++) {
            CHECK(t0[k] <= t1[k] && t1[k] <= t2[k]);
            if (k) CHECK(t1[k] >= t2[k - 1]);
            check_done(s.srv, id[k], *in[k]);
        }
        const frt_server_stats st = stats(s.srv);
        CHECK(st.max_in_flight == 1 && st.completed == 6 && st.failed == 0);
        CHECK(st.bytes_in_use == 0 || st.bytes_in_use == st.peak_bytes || st.bytes_in_use <= st.peak_bytes);
        CHECK(fake::max_batch() == 1);
    }
    end("one_slot_is_fifo", f0);
}

// Slots and the budget bound what is in flight; a request larger than the
// whole budget fails at admission and the others go on.
void slots_and_budget()
{
    const int f0 = g_failures;
    {
        auto probe = make(0, 16, 1);
        const size_t one = bytes_of(*probe);
        Setup s(one * 5 / 2, 3);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        for (int k = 0; k < 10; k++) in.push_back(make(k + 1, 16, 4));
        auto huge = make(99, 40, 2);
        for (auto& i : in) id.push_back(submit(s.srv, *i));
        const uint64_t hid = submit(s.srv, *huge);
        for (size_t k = 0; k < id.size(); k++) check_done(s.srv, id[k], *in[k]);
        check_failed(s.srv, hid, FRT_ENOMEM);
        const frt_server_stats st = stats(s.srv);
        CHECK(st.max_in_flight <= 2);          // two fit the budget, not three
        CHECK(st.peak_bytes <= one * 5 / 2);
        CHECK(st.completed == 10 && st.failed == 1);
    }
    end("slots_and_budget", f0);
}

// Injected failures of one request's creation, upload or step: that request
// fails with the injected code, the others finish with exactly their steps.
void failures_stay_with_their_request()
{
    const int f0 = g_failures;
    for (int mode = 0; mode < 3; mode++) {
        fake::Faults f;
        int code = FRT_ENOMEM;
        if (mode == 0) f.create_fail_at = 3;
        if (mode == 1) f.load_fail_at = 2;
        if (mode == 2) {
            f.step_fail_tag = 4;
            f.step_fail_step = 2;
            f.step_fail_code = code = FRT_EOVERFLOW;
        }
        Setup s(size_t(1) << 40, 8, f);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        for (int k = 0; k < 6; k++) in.push_back(make(k + 1, 12, 5));
        // one at a time up to the failing one, so that the k-th call is known
        for (auto& i : in) {
            id.push_back(submit(s.srv, *i));
            if (mode < 2 && id.size() <= 3) wait_state(s.srv, id.back());
        }
        const size_t bad = mode == 0 ? 2 : mode == 1 ? 1 : 3;
        for (size_t k = 0; k < id.size(); k++) {
            if (k == bad) check_failed(s.srv, id[k], code);
            else check_done(s.srv, id[k], *in[k]);
        }
        const frt_server_stats st = stats(s.srv);
        CHECK(st.completed == 5 && st.failed == 1);
    }
    end("failures_stay_with_their_request", f0);
}

// A device failure fails the whole batch it hit; the server serves on.
void device_failure_fails_its_batch_and_serving_goes_on()
{
    const int f0 = g_failures;
    {
        fake::Faults f;
        f.step_fail_tag = 2;
        f.step_fail_step = 1;
        f.step_fail_code = FRT_EDEVICE;
        Setup s(size_t(1) << 40, 8, f);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        for (int k = 0; k < 4; k++) in.push_back(make(k + 1, 10, 3));
        for (auto& i : in) id.push_back(submit(s.srv, *i));
        int failed = 0;
        for (size_t k = 0; k < id.size(); k++) {
            const int st = wait_state(s.srv, id[k]);
            if (st == FRT_REQ_FAILED) {
                failed++;
                CHECK(frt_server_take(s.srv, id[k], nullptr, nullptr) == FRT_EDEVICE);
            } else {
                check_done(s.srv, id[k], *in[k]);
            }
        }
        CHECK(failed >= 1);
        auto later = make(7, 10, 3);
        check_done(s.srv, submit(s.srv, *later), *later);
    }
    end("device_failure_fails_its_batch_and_serving_goes_on", f0);
}

// Requests that one launch sequence cannot take together (queue mode,
// n_bins) are stepped in separate batches, each request to its end.
void batches_split_by_queue_mode_and_bins()
{
    const int f0 = g_failures;
    {
        Setup s(size_t(1) << 40, 16);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        for (int k = 0; k < 8; k++) in.push_back(make(k + 1, 8 + k, 4, 1 + (k % 2) * 3, (k / 2) % 2 ? 100000 : 0));
        for (auto& i : in) id.push_back(submit(s.srv, *i));
        for (size_t k = 0; k < id.size(); k++) check_done(s.srv, id[k], *in[k]);
        CHECK(stats(s.srv).failed == 0);
    }
    end("batches_split_by_queue_mode_and_bins", f0);
}

// Clients on several threads submit, poll, wait and take at once.
void concurrent_clients()
{
    const int f0 = g_failures;
    {
        Setup s(size_t(1) << 40, 6);
        std::vector<std::thread> th;
        for (int c = 0; c < 4; c++)
            th.emplace_back([&, c] {
                std::vector<std::unique_ptr<Input>> in;
                std::vector<uint64_t> id;
                for (int k = 0; k < 8; k++) {
                    in.push_back(make(100 * (c + 1) + k, 6 + (k % 3) * 4, 2 + k % 4));
                    id.push_back(submit(s.srv, *in.back()));
                    int st;
                    CHECK(frt_server_poll(s.srv, id.back(), &st) == FRT_OK);
                    if (k % 3 == 0) std::this_thread::yield();
                }
                for (size_t k = 0; k < id.size(); k++) check_done(s.srv, id[k], *in[k]);
            });
        for (auto& t : th) t.join();
        const frt_server_stats st = stats(s.srv);
        CHECK(st.completed == 32 && st.failed == 0 && st.max_in_flight <= 6);
        CHECK(st.solve_steps == 4 * (2 * 2 + 3 * 2 + 4 * 2 + 5 * 2));
    }
    end("concurrent_clients", f0);
}

// Destroying the server drops what is queued and running, and frees it.
void destroy_with_requests_in_flight()
{
    const int f0 = g_failures;
    for (int rep = 0; rep < 5; rep++) {
        Setup s(size_t(1) << 40, 4);
        std::vector<std::unique_ptr<Input>> in;
        for (int k = 0; k < 12; k++) {
            in.push_back(make(k + 1, 14, 50));
            submit(s.srv, *in.back());
        }
        if (rep % 2) std::this_thread::yield();
    }
    end("destroy_with_requests_in_flight", f0);
}

// Pass queues bounded by what the budget leaves: two requests admitted
// together whose grown queues do not fit side by side: the batched step
// fails with FRT_ENOMEM and each solve is stepped alone, to its end.
void pass_queue_limit_steps_solves_alone()
{
    const int f0 = g_failures;
    {
        fake::Faults f;
        f.pass_growth = 2;
        auto a = make(1, 16, 30), b = make(2, 16, 3);
        Setup s(2 * bytes_of(*a), 2, f);
        fake::hold_loads(true);
        fake::hold_steps(true);
        const uint64_t ia = submit(s.srv, *a), ib = submit(s.srv, *b);
        wait_admitted(s.srv, {ia, ib}, 2);
        fake::hold_loads(false);
        // both uploads end before the first step does (a step of the first
        // alone may be waiting): the two are in flight together
        for (int k = 0; k < 20000 && fake::loads_done() < 2; k++) std::this_thread::sleep_for(std::chrono::microseconds(500));
        CHECK(fake::loads_done() == 2);
        fake::hold_steps(false);
        check_done(s.srv, ia, *a);
        check_done(s.srv, ib, *b);
        CHECK(fake::max_batch() == 1 && fake::batches() == 33);
        const frt_server_stats st = stats(s.srv);
        CHECK(st.max_in_flight == 2);
        CHECK(st.failed == 0);
        CHECK(st.peak_bytes <= 2 * bytes_of(*a));
    }
    end("pass_queue_limit_steps_solves_alone", f0);
}

// Virtual time: a burst of equal requests served in one batch per tick
// finishes sooner on average than the same burst taken one at a time (each
// launch sequence has a fixed cost besides its per-cell work).
void burst_latency_batched_vs_one_at_a_time()
{
    const int f0 = g_failures;
    double mean[2] = {0, 0};
    for (int m = 0; m < 2; m++) {
        Setup s(size_t(1) << 40, m == 0 ? 1 : 8);
        std::vector<std::unique_ptr<Input>> in;
        std::vector<uint64_t> id;
        for (int k = 0; k < 8; k++) in.push_back(make(k + 1, 8, 10));
        if (m == 1) fake::hold_loads(true);
        for (auto& i : in) id.push_back(submit(s.srv, *i));
        if (m == 1) {
            wait_admitted(s.srv, id, 4);       // four loader threads
            fake::hold_loads(false);
        }
        for (size_t k = 0; k < id.size(); k++) {
            CHECK(wait_state(s.srv, id[k]) == FRT_REQ_DONE);
            double t[3];
            CHECK(frt_server_times(s.srv, id[k], t) == FRT_OK);
            mean[m] += (t[2] - t[0]) / (double)id.size();
            check_done(s.srv, id[k], *in[k]);
        }
        if (m == 1) CHECK(fake::max_batch() >= 2);
    }
    std::printf("burst of 8: mean latency %.3e s one at a time, %.3e s batched (virtual time)\n", mean[0], mean[1]);
    CHECK(mean[1] < mean[0]);
    end("burst_latency_batched_vs_one_at_a_time", f0);
}

// A request with the temperature on hands back its T before it is taken; one
// without it, an unfinished one and a taken one do not.
void temperature_is_read_before_take()
{
    const int f0 = g_failures;
    Setup S(size_t(1) << 30, 4);
    auto warm = make(5.0, 6, 3);
    warm->r.params.temperature = 1;
    auto cold = make(6.0, 6, 3);
    fake::hold_steps(true);
    const uint64_t a = submit(S.srv, *warm), b = submit(S.srv, *cold);
    std::vector<double> T(warm->ncell);
    CHECK(frt_server_read_temperature(S.srv, a, T.data()) == FRT_ESTATE);   // not finished
    fake::hold_steps(false);
    CHECK(wait_state(S.srv, a) == FRT_REQ_DONE);
    CHECK(wait_state(S.srv, b) == FRT_REQ_DONE);
    CHECK(frt_server_read_temperature(S.srv, a, T.data()) == FRT_OK);
    const size_t probe[3] = {0, warm->ncell / 2, warm->ncell - 1};
    for (size_t k : probe) CHECK(T[k] == fake::expected_T(5.0, 3, k));
    CHECK(frt_server_read_temperature(S.srv, b, T.data()) == FRT_ESTATE);   // no temperature
    CHECK(frt_server_read_temperature(S.srv, a, nullptr) == FRT_EINVAL);
    check_done(S.srv, a, *warm);
    check_done(S.srv, b, *cold);
    CHECK(frt_server_read_temperature(S.srv, a, T.data()) == FRT_EINVAL);   // taken: forgotten
    end("temperature_is_read_before_take", f0);
}

}  // namespace

int main()
{
    one_slot_is_fifo();
    slots_and_budget();
    failures_stay_with_their_request();
    device_failure_fails_its_batch_and_serving_goes_on();
    batches_split_by_queue_mode_and_bins();
    concurrent_clients();
    destroy_with_requests_in_flight();
    pass_queue_limit_steps_solves_alone();
    burst_latency_batched_vs_one_at_a_time();
    temperature_is_read_before_take();
    std::printf("%s: %d failed checks\n", g_failures ? "FAILED" : "all scenarios passed", g_failures);
    return g_failures > 255 ? 255 : g_failures;
}
