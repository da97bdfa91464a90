// fdtd_step_static: the time stepping of fdtd_step for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc). The only scratch the step kernels use, the
// per-workgroup partial sums of the energy diagnostic, lives in a
// file-scope device array here instead of a context buffer; everything
// else a step touches (fields, CPML memories, tables, plane sums, the
// energy result) already belongs to the context. Nothing is allocated,
// freed or created: no streams, no events (the boundary launches of the
// two-step kernel run on the caller's stream, after the interior's), no
// profiling marks, no growth of the time tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "context.hpp"

using namespace bfdtd;

namespace {

// 2 MiB: the energy partials of a 768 x 768 x 255 grid at the default tile
// take about 156 K of them.
constexpr int kScratchDoubles = 1 << 18;
__device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device, taken once per device with
// that device current. In host code the name `scratch` is only a host-side
// stand-in: every kernel argument and fill uses the address kept here.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

double* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    need(dev >= 0 && dev < kMaxDevices, "device index out of range");
    if (!g_scratch[dev]) {
        void* p = nullptr;
        check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        need(p != nullptr, "no device address for the static scratch", FDTD_EDEVICE);
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

__global__ void __launch_bounds__(256) zero_fill(double* p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0.0;
}

// Makes the context's device current for the call and restores the
// caller's afterwards.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Detaches the profiler (whose marks create events) for the call.
struct NoTimer {
    fdtd_ctx* c;
    EventTimer* t;
    explicit NoTimer(fdtd_ctx* ctx) : c(ctx), t(ctx->timer) { ctx->timer = nullptr; }
    ~NoTimer() { c->timer = t; }
};

}  // namespace

extern "C" int fdtd_step_static(fdtd_ctx* c, int64_t nsteps) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(nsteps >= 0, "nsteps must be >= 0");
        if (nsteps == 0) return;
        DeviceScope dev(c->device);
        NoTimer nt(c);
        if (c->has_inj) {
            char buf[160];
            std::snprintf(buf, sizeof buf,
                          "the time tables reach step %lld; this call needs %lld "
                          "(fdtd_step grows them)",
                          c->t_cap, (long long)(c->step + nsteps));
            need(c->step + nsteps <= c->t_cap, buf, FDTD_ESTATE);
        }
        if (frame_fused(c)) {
            const Frame fr = interior_of(c);
            const int cz = std::min(frame_cz(c), c->p.nz);
            need(c->ftiles && cz == c->fcz && c->frame_rows == c->frows &&
                     fr.x0 == c->ftile_rect.x0 && fr.x1 == c->ftile_rect.x1 &&
                     fr.y0 == c->ftile_rect.y0 && fr.y1 == c->ftile_rect.y1,
                 "the fused frame's tile list is not built for this tile; run fdtd_step once",
                 FDTD_ESTATE);
        }
        const bool energy = (c->mask & FDTD_DIAG_ENERGY) != 0;
        const bool pairs = two_step_on(c), triples = three_step_on(c);
        int np = 0;
        double* part = nullptr;
        if (energy) {
            np = std::max(1, partial_count(c));
            char buf[160];
            std::snprintf(buf, sizeof buf,
                          "the energy diagnostic needs %d partial sums here; the static "
                          "scratch holds %d",
                          np, kScratchDoubles);
            need(np <= kScratchDoubles, buf);
            part = scratch_on(c->device);
        }
        for (int64_t s = 0; s < nsteps;) {
            const long long n = c->step;
            if (triples && nsteps - s >= 3) {
                Problem q = c->p;
                q.plane = c->plane;
                const unsigned dm = c->mask & 7u;
                const int m0 = (c->plane >= 0 && n >= c->wbegin) ? (int)dm : 0;
                const int m1 = (c->plane >= 0 && n + 1 >= c->wbegin) ? (int)dm : 0;
                const int m2 = (c->plane >= 0 && n + 2 >= c->wbegin) ? (int)dm : 0;
                check(launch_step3(q, n, c->parity, c->tb_rows, c->tb_zchunk, m0, m1, m2,
                                   c->stream, nullptr, nullptr),
                      "three-step launch");
                c->count += (m0 != 0) + (m1 != 0) + (m2 != 0);
                c->parity ^= 1;
                c->step += 3;
                s += 3;
                continue;
            }
            if (pairs && nsteps - s >= 2) {
                Problem q = c->p;
                q.plane = c->plane;
                const unsigned dm = c->mask & 7u;
                const int m0 = (c->plane >= 0 && n >= c->wbegin) ? (int)dm : 0;
                const int m1 = (c->plane >= 0 && n + 1 >= c->wbegin) ? (int)dm : 0;
                check(launch_step2(q, n, c->parity, c->tb_rows, c->tb_zchunk, m0, m1, c->stream,
                                   nullptr, nullptr),
                      "two-step launch");
                c->count += (m0 != 0) + (m1 != 0);
                c->parity ^= 1;
                c->step += 2;
                s += 2;
                continue;
            }
            Problem q = c->p;
            const bool in_window = c->plane >= 0 && n >= c->wbegin;
            q.diag_mask = in_window ? (int)(c->mask & 7u) : 0;
            q.plane = c->plane;
            if (part) {
                // the scratch keeps the last call's contents (another context's
                // included): slots a step does not write must read zero
                hipLaunchKernelGGL(zero_fill, dim3(std::min((np + 255) / 256, 1024)), dim3(256),
                                   0, c->stream, part, np);
                check(hipGetLastError(), "zero fill");
            }
            check(launch_step(c, q, n, c->parity, part), "step launch");
            if (part) {
                check(launch_energy_reduce(part, np, c->energy_dev, c->stream), "energy reduce");
                c->energy_valid = true;
            }
            if (q.diag_mask) c->count += 1;
            c->parity ^= 1;
            c->step += 1;
            s += 1;
        }
    });
}
