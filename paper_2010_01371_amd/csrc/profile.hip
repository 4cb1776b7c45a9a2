// Optional per-kernel timing with HIP events recorded on the launch stream.
//
// When enabled (mbmd_profile_enable), every instrumented launch is bracketed
// by a pair of hipEvents on the stream it is launched on; mbmd_profile_query
// waits for them and reports the number of launches and their summed
// duration per kernel name.  Launches enqueued while a stream is being
// captured into a graph are not instrumented.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace mbmd {

namespace {
struct Pending {
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, std::vector<Pending>> g_pending;
std::map<std::string, std::pair<long long, double>> g_done;   // launches, ms
std::vector<hipEvent_t> g_pool;
std::string g_select;                // empty: every kernel; else ",name1,name2,"

bool selected(const char* name) {
    if (g_select.empty()) return true;
    return g_select.find("," + std::string(name) + ",") != std::string::npos;
}

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    MBMD_HIP(hipEventCreate(&e));
    return e;
}

void resolve_locked() {
    for (auto& kv : g_pending) {
        auto& done = g_done[kv.first];
        for (auto& p : kv.second) {
            MBMD_HIP(hipEventSynchronize(p.b));
            float ms = 0.0f;
            MBMD_HIP(hipEventElapsedTime(&ms, p.a, p.b));
            done.first += 1;
            done.second += ms;
            g_pool.push_back(p.a);
            g_pool.push_back(p.b);
        }
        kv.second.clear();
    }
}
}  // namespace

namespace {
// Kernels with a batched form (they shift their pointers by the slice offsets).
bool batched_form(const char* name) {
    static const char* const names[] = {"k_ray_grad", "k_curvature", "k_line_prefix", "k_dd_forward",
                                        "k_detector_prefix", "k_dd_back", "k_penalty_grad", "k_fft_rows_fwd",
                                        "k_fft_cols", "k_fft_rows_inv", "k_reduce_final", "k_axpy2_alpha",
                                        "k_fill_double", "k_block_apply", "k_dot", "k_plain_update", "k_fill",
                                        "k_add_part", "k_scale_copy", "k_haar_fwd_tile", "k_haar_coarse_fwd",
                                        "k_haar_coarse_inv", "k_haar_inv_tile", "k_d4_pass", "k_d4_coarse",
                                        "k_ray_means", "k_blur_resid", "k_ray_grad_r"};
    for (const char* n : names)
        if (std::strcmp(n, name) == 0) return true;
    return false;
}
}  // namespace

ZBatch& zbatch() {
    static thread_local ZBatch z;
    return z;
}

KernelTimer::KernelTimer(const char* name, hipStream_t s) : name_(name), s_(s) {
    MBMD_REQUIRE(zbatch().zd == nullptr || batched_form(name), MBMD_ERR_UNSUPPORTED,
                 std::string("no batched form of ") + name);
    if (!g_on) return;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!selected(name)) return;
    }
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lock(g_mu);
    a_ = get_event();
    b_ = get_event();
    MBMD_HIP(hipEventRecord(a_, s_));
    active_ = true;
}

void KernelTimer::stop() {
    if (!active_) return;
    std::lock_guard<std::mutex> lock(g_mu);
    MBMD_HIP(hipEventRecord(b_, s_));
    g_pending[name_].push_back(Pending{a_, b_});
    if (g_pending[name_].size() > 4096) resolve_locked();
    active_ = false;
}

}  // namespace mbmd

using namespace mbmd;

extern "C" {

int mbmd_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_on = on != 0;
    return MBMD_OK;
}

int mbmd_profile_select(const char* names) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_select = (names && *names) ? "," + std::string(names) + "," : std::string();
    return MBMD_OK;
}

int mbmd_profile_reset(void) {
    try {
        std::lock_guard<std::mutex> lock(g_mu);
        resolve_locked();
        g_done.clear();
        return MBMD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    }
}

int mbmd_profile_query(const char* kernel, long long* launches, double* total_ms) {
    if (!kernel || !launches || !total_ms) return MBMD_ERR_ARG;
    try {
        std::lock_guard<std::mutex> lock(g_mu);
        resolve_locked();
        auto it = g_done.find(kernel);
        *launches = it == g_done.end() ? 0 : it->second.first;
        *total_ms = it == g_done.end() ? 0.0 : it->second.second;
        return MBMD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    }
}

int mbmd_profile_kernels(char* names, size_t capacity) {
    if (!names || capacity == 0) return MBMD_ERR_ARG;
    try {
        std::lock_guard<std::mutex> lock(g_mu);
        resolve_locked();
        std::string all;
        for (auto& kv : g_done) {
            if (!all.empty()) all += ",";
            all += kv.first;
        }
        if (all.size() + 1 > capacity) return MBMD_ERR_ARG;
        std::memcpy(names, all.c_str(), all.size() + 1);
        return MBMD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    }
}

}  // extern "C"
