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
    // the record each stream has open (the event recorded next on that
    // stream closes it)
    std::vector<std::pair<hipStream_t, int>> pending;
    void mark(const char* name) override { mark_on(name, stream); }
    void mark_on(const char* name, hipStream_t s) override {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, s);
        bool used = false;
        int* slot = nullptr;
        for (auto& q : pending)
            if (q.first == s) slot = &q.second;
        if (!slot) {
            pending.push_back({s, -1});
            slot = &pending.back().second;
        }
        if (*slot >= 0) {
            open_[*slot].b = e;
            used = true;
        }
        *slot = -1;
        if (name) {
            open_.push_back(Rec{name, e, nullptr});
            *slot = (int)open_.size() - 1;
            used = true;
        }
        if (!used) (void)hipEventDestroy(e);
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
        pending.clear();
    }
    ~EventTimer() override { collect(); }
};

struct fdtd_ctx {
    fdtd_grid g{};
    hipStream_t stream = nullptr;
    int device = 0;
    double ry = 1, rz = 1;
    bfdtd::Problem p{};
    std::vector<std::pair<void*, size_t>> allocs;   // device buffers and their bytes
    long long device_bytes = 0;                      // sum of the bytes in allocs
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
    // frame around the fused interior: split kernels, or fused boundary tiles
    int frame = FDTD_FRAME_SPLIT;
    int xalign = 32;                // interior x origin multiple (32 or 64 cells)
    int frame_rows = 2;             // rows per fused frame tile (2 or 4)
    int4* ftiles = nullptr;         // fused frame tiles (0, x0, y0, z chunk)
    int nftiles = 0, ftile_cap = 0, fblocks = 0, fcz = 0, frows = 0;
    bfdtd::Frame ftile_rect{0, 0, 0, 0};
    // steps per pass over the fields (time_block 2: the two-step kernel, 3:
    // the three-step kernel, with pairs and single steps for the rest)
    int time_block = 1, tb_rows = 4, tb_zchunk = 0;
    bfdtd::SideStreams side{};     // the two-step kernel's boundary launches
    bool side_ok = false;
    bool concurrent = true;        // boundary launches beside the interior (else in order)
    bool batch_owned = false;      // stepped by an fdtd_batch
    // bumped by every change of the antenna or its sector weights: an
    // adjoint's reverse sweep refuses to run on checkpoints of another antenna
    long long inj_version = 0;
    std::vector<fdtd_adjoint*> adjoints;   // attached adjoints (detached on destroy)
    EventTimer* timer = nullptr;
    std::string err;
};

namespace bfdtd {

// Called by fdtd_destroy for each attached adjoint: the adjoint forgets its
// forward context (its calls then fail with FDTD_ESTATE) and can still be
// destroyed.
void detach_adjoint(fdtd_adjoint* a);

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
    c->allocs.emplace_back(ptr, count * sizeof(T));
    c->device_bytes += (long long)(count * sizeof(T));
    check(hipMemsetAsync(ptr, 0, count * sizeof(T), c->stream), "hipMemsetAsync");
    return static_cast<T*>(ptr);
}

inline void dfree(fdtd_ctx* c, void* ptr) {
    if (!ptr) return;
    auto it = std::find_if(c->allocs.begin(), c->allocs.end(),
                           [ptr](const std::pair<void*, size_t>& a) { return a.first == ptr; });
    if (it != c->allocs.end()) {
        c->device_bytes -= (long long)it->second;
        c->allocs.erase(it);
    }
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

// A fused step: the interior kernel, then the frame around it, either by the
// split kernels (the whole grid when there is no interior or for the split
// kernel choice) or by one launch of the fused boundary-tile kernel.
inline Frame interior_of(const fdtd_ctx* c) {
    if (c->kernel == FDTD_KERNEL_SPLIT) return Frame{0, 0, 0, 0};
    return fused_interior_rect(c->p, c->rows, c->xalign);
}

// (the fused boundary tiles know walls and CPML but not the periodic test mode)
inline bool frame_fused(const fdtd_ctx* c) {
    return c->kernel != FDTD_KERNEL_SPLIT && c->frame == FDTD_FRAME_FUSED && !c->p.periodic;
}

inline int interior_partials(const fdtd_ctx* c) {
    return c->kernel == FDTD_KERNEL_SPLIT ? 0
                                          : fused_interior_tiles(c->p, c->rows, c->zchunk, c->xalign);
}

inline int frame_cz(const fdtd_ctx* c) { return c->zchunk > 0 ? c->zchunk : 16; }

inline int partial_count(const fdtd_ctx* c) {
    const int fp = frame_fused(c) ? c->nftiles : split_partial_count(c->p, interior_of(c));
    return interior_partials(c) + fp;
}

// Tile list of the fused frame: every 64 x frame_rows tile (x0 a multiple of
// 64, y0 of frame_rows) that holds a grid cell outside the interior, per z
// chunk.
inline void ensure_frame_tiles(fdtd_ctx* c) {
    if (!frame_fused(c)) return;
    const Frame fr = interior_of(c);
    const int cz = std::min(frame_cz(c), c->p.nz);
    const int rows = c->frame_rows;
    if (c->ftiles && cz == c->fcz && rows == c->frows && fr.x0 == c->ftile_rect.x0 &&
        fr.x1 == c->ftile_rect.x1 &&
        fr.y0 == c->ftile_rect.y0 && fr.y1 == c->ftile_rect.y1)
        return;
    const Problem& p = c->p;
    std::vector<int4> t;
    for (int ch = 0; ch * cz < p.nz; ++ch)
        for (int y0 = 0; y0 < p.ny; y0 += rows)
            for (int x0 = 0; x0 < p.nx; x0 += 64) {
                const bool inside = x0 >= fr.x0 && x0 + 64 <= fr.x1 && y0 >= fr.y0 &&
                                    y0 + rows <= fr.y1;
                if (!inside) t.push_back(make_int4(0, x0, y0, ch));
            }
    check(hipStreamSynchronize(c->stream), "sync");   // the old list may be in use
    if ((int)t.size() > c->ftile_cap) {
        dfree(c, c->ftiles);
        c->ftiles = dalloc<int4>(c, t.size());
        c->ftile_cap = (int)t.size();
    }
    check(hipMemcpy(c->ftiles, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice),
          "copy frame tiles");
    c->nftiles = (int)t.size();
    c->fcz = cz;
    c->frows = rows;
    c->ftile_rect = fr;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    c->fblocks = std::max(1, std::min((c->nftiles + 3) / 4, cus * fused_bnd_blocks_per_cu(rows, false)));
}

inline void ensure_partials(fdtd_ctx* c) {
    ensure_frame_tiles(c);
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
        hipError_t e = launch_fused_interior(q, n, parity, c->rows, c->zchunk, c->xalign, epart,
                                             c->stream, c->timer);
        if (e != hipSuccess) return e;
        off = interior_partials(c);
    }
    if (frame_fused(c)) {
        if (c->timer) c->timer->mark("frame_fused");
        hipError_t e = launch_fused_bnd(q, nullptr, c->ftiles, c->nftiles, c->frows, c->fcz,
                                        c->fblocks, nullptr, n, parity, 1, fr,
                                        epart ? epart + off : nullptr, c->stream);
        if (c->timer) c->timer->mark(nullptr);
        return e;
    }
    return launch_split_frame(q, n, parity, fr, epart ? epart + off : nullptr, c->stream,
                              c->timer);
}

// Pairs of steps go through the two-step kernel when it (or the
// three-step kernel) is selected, the fused kernel is in use, the walls are
// not periodic, and neither the energy record nor a plane record is wanted
// (those need every step's state); triples go through the three-step kernel
// under the same conditions when it is selected.
inline bool two_step_on(const fdtd_ctx* c) {
    return (c->time_block == 2 || c->time_block == 3) && c->kernel != FDTD_KERNEL_SPLIT &&
           !c->p.periodic && !(c->mask & FDTD_DIAG_ENERGY) && !c->p.rec;
}
inline bool three_step_on(const fdtd_ctx* c) {
    return c->time_block == 3 && two_step_on(c);
}

// Steps n and n + 1 in one pass over the whole grid: the two-step kernel
// reads the fields and CPML memories of parity par and writes those of
// parity par ^ 1.
// trial: a timing run that leaves the state alone (it writes only parity
// par ^ 1; no plane sums, and the step count does not move).
inline void create_side_streams(SideStreams& q) {
    q = SideStreams{};
    for (int i = 0; i < 3; ++i) {
        check(hipStreamCreateWithFlags(&q.s[i], hipStreamNonBlocking), "side stream");
        check(hipEventCreateWithFlags(&q.join[i], hipEventDisableTiming), "side event");
    }
    check(hipEventCreateWithFlags(&q.fork, hipEventDisableTiming), "side event");
}

inline void release_side_streams(SideStreams& q) {
    for (int i = 0; i < 3; ++i) {
        if (q.s[i]) (void)hipStreamDestroy(q.s[i]);
        if (q.join[i]) (void)hipEventDestroy(q.join[i]);
    }
    if (q.fork) (void)hipEventDestroy(q.fork);
    q = SideStreams{};
}

inline void ensure_side_streams(fdtd_ctx* c) {
    if (c->side_ok) return;
    try {
        create_side_streams(c->side);
    } catch (...) {
        release_side_streams(c->side);
        throw;
    }
    c->side_ok = true;
}

inline void destroy_side_streams(fdtd_ctx* c) {
    if (!c->side_ok) return;
    release_side_streams(c->side);
    c->side_ok = false;
}

inline void launch_pair(fdtd_ctx* c, long long n, bool trial = false) {
    const int par = c->parity;
    Problem q = c->p;
    q.plane = c->plane;
    const unsigned dm = trial ? 0u : c->mask & 7u;
    const int m0 = (c->plane >= 0 && n >= c->wbegin) ? (int)dm : 0;
    const int m1 = (c->plane >= 0 && n + 1 >= c->wbegin) ? (int)dm : 0;
    if (c->concurrent) ensure_side_streams(c);
    check(launch_step2(q, n, par, c->tb_rows, c->tb_zchunk, m0, m1, c->stream, c->timer,
                       c->concurrent ? &c->side : nullptr),
          "two-step launch");
    if (trial) return;
    c->count += (m0 != 0) + (m1 != 0);
    c->parity ^= 1;
    c->step += 2;
}

// Steps n .. n + 2 in one pass over the whole grid through the three-step
// kernel (parity par to par ^ 1); trial as for launch_pair.
inline void launch_triple(fdtd_ctx* c, long long n, bool trial = false) {
    const int par = c->parity;
    Problem q = c->p;
    q.plane = c->plane;
    const unsigned dm = trial ? 0u : c->mask & 7u;
    const int m0 = (c->plane >= 0 && n >= c->wbegin) ? (int)dm : 0;
    const int m1 = (c->plane >= 0 && n + 1 >= c->wbegin) ? (int)dm : 0;
    const int m2 = (c->plane >= 0 && n + 2 >= c->wbegin) ? (int)dm : 0;
    if (c->concurrent) ensure_side_streams(c);
    check(launch_step3(q, n, par, c->tb_rows, c->tb_zchunk, m0, m1, m2, c->stream, c->timer,
                       c->concurrent ? &c->side : nullptr),
          "three-step launch");
    if (trial) return;
    c->count += (m0 != 0) + (m1 != 0) + (m2 != 0);
    c->parity ^= 1;
    c->step += 3;
}

}  // namespace bfdtd
