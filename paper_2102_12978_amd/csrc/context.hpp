// Host-side state of one solver context and the error/allocation helpers
// shared by the single-domain C ABI (capi.cpp) and the batch (batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "fdtd_internal.hpp"

// Event-pair timer for fdtd_profile_*: one event before each launch, the
// next mark closes it.
struct EventTimer : bfdtd::LaunchTimer {
    hipStream_t stream = nullptr;
    struct Rec {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Rec> open_;
    std::vector<std::pair<std::string, std::pair<long long, double>>> totals;
    int pending = -1;
    void mark(const char* name) override {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, stream);
        if (pending >= 0) open_[pending].b = e;
        pending = -1;
        if (name) {
            open_.push_back(Rec{name, e, nullptr});
            pending = (int)open_.size() - 1;
        } else if (open_.empty() || open_.back().b != e) {
            (void)hipEventDestroy(e);
        }
    }
    void collect() {
        std::vector<hipEvent_t> seen;
        for (auto& r : open_) {
            if (!r.b) continue;
            (void)hipEventSynchronize(r.b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            bool found = false;
            for (auto& t : totals)
                if (t.first == r.name) {
                    t.second.first += 1;
                    t.second.second += ms;
                    found = true;
                }
            if (!found) totals.push_back({r.name, {1, (double)ms}});
        }
        for (auto& r : open_) {
            for (hipEvent_t e : {r.a, r.b}) {
                if (!e) continue;
                if (std::find(seen.begin(), seen.end(), e) == seen.end()) {
                    seen.push_back(e);
                    (void)hipEventDestroy(e);
                }
            }
        }
        open_.clear();
        pending = -1;
    }
    ~EventTimer() override { collect(); }
};

struct fdtd_ctx {
    fdtd_grid g{};
    hipStream_t stream = nullptr;
    int device = 0;
    double ry = 1, rz = 1;
    bfdtd::Problem p{};
    std::vector<void*> allocs;
    long long device_bytes = 0;
    // antenna
    bool has_inj = false;
    bfdtd::Antenna ant;
    int* colmap = nullptr;
    float2* amp = nullptr;
    float2* zph = nullptr;
    float2* tE = nullptr;
    float2* tH = nullptr;
    long long t_cap = 0;
    // diagnostics
    int plane = -1;
    long long wbegin = 0;
    unsigned mask = 0;
    long long count = 0;
    double* fl = nullptr;
    double* epart = nullptr;
    int epart_cap = 0;
    double* energy_dev = nullptr;
    bool energy_valid = false;
    // stepping
    long long step = 0;
    int parity = 0;
    int kernel = FDTD_KERNEL_FUSED;
    int rows = 4, zchunk = 0;
    bool batch_owned = false;      // stepped by an fdtd_batch
    EventTimer* timer = nullptr;
    std::string err;
};

namespace bfdtd {

struct Fail {
    int code;
    std::string msg;
};

inline void check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FDTD_ENOMEM
                                                                              : FDTD_EDEVICE;
        throw Fail{code, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

template <typename T>
T* dalloc(fdtd_ctx* c, size_t count) {
    if (count == 0) return nullptr;
    void* ptr = nullptr;
    check(hipMalloc(&ptr, count * sizeof(T)), "hipMalloc");
    c->allocs.push_back(ptr);
    c->device_bytes += (long long)(count * sizeof(T));
    check(hipMemsetAsync(ptr, 0, count * sizeof(T), c->stream), "hipMemsetAsync");
    return static_cast<T*>(ptr);
}

inline void dfree(fdtd_ctx* c, void* ptr) {
    if (!ptr) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), ptr);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(ptr);
}

template <typename F>
int guarded(fdtd_ctx* c, F&& f) {
    try {
        f();
        return FDTD_OK;
    } catch (const Fail& e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return FDTD_ENOMEM;
    } catch (...) {
        if (c) c->err = "unexpected exception";
        return FDTD_EDEVICE;
    }
}

inline void need(bool ok, const std::string& msg, int code = FDTD_EINVAL) {
    if (!ok) throw Fail{code, msg};
}

inline void ensure_time_tables(fdtd_ctx* c, long long upto) {
    if (!c->has_inj || upto <= c->t_cap) return;
    check(hipStreamSynchronize(c->stream), "sync");   // old tables may be in use
    long long cap = std::max(upto, std::max(2 * c->t_cap, 1024LL));
    std::vector<float2> te(cap), th(cap);
    const double dt = c->g.courant;
    for (long long n = 0; n < cap; ++n) {
        double re, im;
        time_factor(c->ant, (n + 1.0) * dt, &re, &im);
        te[n] = make_float2((float)re, (float)im);
        time_factor(c->ant, (n + 1.5) * dt, &re, &im);
        th[n] = make_float2((float)re, (float)im);
    }
    dfree(c, c->tE);
    dfree(c, c->tH);
    c->tE = dalloc<float2>(c, cap);
    c->tH = dalloc<float2>(c, cap);
    check(hipMemcpyAsync(c->tE, te.data(), cap * sizeof(float2), hipMemcpyHostToDevice, c->stream),
          "copy time table");
    check(hipMemcpyAsync(c->tH, th.data(), cap * sizeof(float2), hipMemcpyHostToDevice, c->stream),
          "copy time table");
    check(hipStreamSynchronize(c->stream), "sync");
    c->t_cap = cap;
    c->p.tE = c->tE;
    c->p.tH = c->tH;
}

// A fused step: the interior kernel, then the split kernels on the frame
// around it (the whole grid when there is no interior or for the split
// kernel choice).
inline Frame interior_of(const fdtd_ctx* c) {
    if (c->kernel == FDTD_KERNEL_SPLIT) return Frame{0, 0, 0, 0};
    return fused_interior_rect(c->p, c->rows);
}

inline int interior_partials(const fdtd_ctx* c) {
    return c->kernel == FDTD_KERNEL_SPLIT ? 0 : fused_interior_tiles(c->p, c->rows, c->zchunk);
}

inline int partial_count(const fdtd_ctx* c) {
    return interior_partials(c) + split_partial_count(c->p, interior_of(c));
}

inline void ensure_partials(fdtd_ctx* c) {
    int need_n = std::max(1, partial_count(c));
    if (need_n <= c->epart_cap) return;
    check(hipStreamSynchronize(c->stream), "sync");
    dfree(c, c->epart);
    c->epart = dalloc<double>(c, need_n);
    c->epart_cap = need_n;
}

inline hipError_t launch_step(const fdtd_ctx* c, const Problem& q, long long n, int parity,
                       double* epart) {
    const Frame fr = interior_of(c);
    int off = 0;
    if (fr.x1 > fr.x0) {
        hipError_t e = launch_fused_interior(q, n, parity, c->rows, c->zchunk, epart, c->stream,
                                             c->timer);
        if (e != hipSuccess) return e;
        off = interior_partials(c);
    }
    return launch_split_frame(q, n, parity, fr, epart ? epart + off : nullptr, c->stream,
                              c->timer);
}

}  // namespace bfdtd
