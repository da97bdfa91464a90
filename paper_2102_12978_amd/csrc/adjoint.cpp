// Reverse-mode gradient of a time-averaged intensity loss with respect to
// the antenna's sector weights: forward run with state checkpoints, then a
// reverse sweep of transposed steps (kernels_adjoint.hip) that recomputes,
// segment by segment from the checkpoints, the E_y planes the loss needs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "context.hpp"

using namespace bfdtd;

namespace bfdtd {
hipError_t launch_adjoint_h(const Problem& lam, int par, const Frame& fr, hipStream_t s);
hipError_t launch_adjoint_e(const Problem& lam, int par, const Frame& fr, hipStream_t s);
hipError_t launch_adjoint_inject(const Problem& lam, int par, const float* g, const float* ey,
                                 float coef, hipStream_t s);
hipError_t launch_adjoint_gacc(const Problem& lam, int par_h, int par_e, const int* slot_i,
                               const int* slot_j, int nslots, float2 tH, float2 tE, double2* G,
                               hipStream_t s);
}  // namespace bfdtd

struct fdtd_adjoint {
    fdtd_ctx* c = nullptr;
    int every = 100;                    // checkpoint interval (steps)
    Problem lam{};                      // λ: fields and ψ ping-pong, like the forward state
    int lam_par = 0;                    // parity of the current λ
    std::vector<std::pair<void*, size_t>> allocs;   // device buffers and their bytes
    long long device_bytes = 0;                      // sum of the bytes in allocs
    // checkpoints of the forward state after s * every steps
    std::vector<float*> ck_f, ck_psi;
    std::vector<int> ck_par;
    long long nsteps = 0, wbegin = 0;
    int plane = -1;
    bool have_forward = false;
    float* rec = nullptr;               // E_y planes of one segment [every][ny][nx]
    float* g_dev = nullptr;             // ∂L/∂Ī [ny][nx]
    double2* G = nullptr;               // [slot][6]
    int* slot_i = nullptr;
    int* slot_j = nullptr;
    int nslots = 0;
    long long recompute_steps = 0;
    long long inj_version = -1;         // forward context's antenna version at the forward run
    long long runs = 0;                 // completed fdtd_adjoint_forward calls
    std::string err;
};

namespace bfdtd {
void detach_adjoint(fdtd_adjoint* a) { a->c = nullptr; }
}  // namespace bfdtd

namespace {

thread_local std::string g_adj_create_error;

template <typename F>
int aguard(fdtd_adjoint* a, F&& f) {
    try {
        f();
        return FDTD_OK;
    } catch (const Fail& e) {
        if (a) a->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (a) a->err = "host allocation failed";
        return FDTD_ENOMEM;
    } catch (...) {
        if (a) a->err = "unexpected exception";
        return FDTD_EDEVICE;
    }
}

void attached(const fdtd_adjoint* a) {
    need(a->c != nullptr, "the forward context was destroyed", FDTD_ESTATE);
}

template <typename T>
T* aalloc(fdtd_adjoint* a, size_t count) {
    void* p = nullptr;
    check(hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)), "hipMalloc");
    a->allocs.emplace_back(p, std::max<size_t>(1, count) * sizeof(T));
    a->device_bytes += (long long)(std::max<size_t>(1, count) * sizeof(T));
    return static_cast<T*>(p);
}

void afree(fdtd_adjoint* a, void* p) {
    if (!p) return;
    auto it = std::find_if(a->allocs.begin(), a->allocs.end(),
                           [p](const std::pair<void*, size_t>& q) { return q.first == p; });
    if (it != a->allocs.end()) {
        a->device_bytes -= (long long)it->second;
        a->allocs.erase(it);
    }
    (void)hipFree(p);
}

size_t field_bytes(const Problem& p) { return 6 * field_elems(p) * sizeof(float); }
size_t psi_bytes(const Problem& p) { return p.npml > 0 ? psi_total(p) * sizeof(float) : 0; }

void clear_lambda(fdtd_adjoint* a) {
    hipStream_t s = a->c->stream;
    for (int par = 0; par < 2; ++par) {
        check(hipMemsetAsync(a->lam.fbase[par], 0, field_bytes(a->lam), s), "clear");
        if (psi_bytes(a->lam)) check(hipMemsetAsync(a->lam.pbase[par], 0, psi_bytes(a->lam), s), "clear");
    }
    a->lam_par = 0;
}

// The λ problem shares the forward tables (CPML, antenna, time) and sizes.
void sync_lambda_tables(fdtd_adjoint* a) {
    const Problem& f = a->c->p;
    Problem& l = a->lam;
    l.ctab = f.ctab;
    l.colmap = f.colmap;
    l.amp = f.amp;
    l.zph = f.zph;
    l.tE = f.tE;
    l.tH = f.tH;
    l.plane = a->plane;
}

float2 time_value(const fdtd_ctx* c, double steps);

// One transposed step, λ of parity par -> par ^ 1. On the interior of the
// forward context's fused kernel the transposed step is the forward Yee
// step with S_x, S_y, S_z negated and no source (the Yee curls are each
// other's transposes), so the fused interior kernel runs it there; the
// transposed-CPML kernels take the frame (the whole grid for the split
// kernel choice or the periodic test mode). With correlations, G picks up
// the H components of λ as they were before the step (parity par, left
// intact) and the E components after its H-part transpose (final in
// parity par ^ 1), in one launch after the step.
void reverse_step(fdtd_adjoint* a, bool correlate, long long m) {
    fdtd_ctx* c = a->c;
    hipStream_t s = c->stream;
    const int par = a->lam_par;
    Frame fr{0, 0, 0, 0};
    if (c->kernel != FDTD_KERNEL_SPLIT && !a->lam.periodic) {
        fr = fused_interior_rect(a->lam, c->rows, c->xalign);
        if (fr.x1 > fr.x0) {
            Problem q = a->lam;
            q.sx = -q.sx;
            q.sy = -q.sy;
            q.sz = -q.sz;
            q.colmap = nullptr;
            q.fl = nullptr;
            q.rec = nullptr;
            q.diag_mask = 0;
            q.plane = -1;
            check(launch_fused_interior(q, 0, par, c->rows, c->zchunk, c->xalign, nullptr, s,
                                        nullptr), "adjoint interior launch");
        }
    }
    check(launch_adjoint_h(a->lam, par, fr, s), "adjoint H launch");
    check(launch_adjoint_e(a->lam, par, fr, s), "adjoint E launch");
    if (correlate)
        check(launch_adjoint_gacc(a->lam, par, par ^ 1, a->slot_i, a->slot_j, a->nslots,
                                  time_value(c, m + 1.5), time_value(c, m + 1.0), a->G, s),
              "G");
    a->lam_par ^= 1;
}

void transposed_step(fdtd_adjoint* a) {   // source-free, no loss term
    reverse_step(a, false, 0);
}

void save_checkpoint(fdtd_adjoint* a, int q) {
    fdtd_ctx* c = a->c;
    const Problem& p = c->p;
    if ((int)a->ck_f.size() <= q) {
        a->ck_f.push_back(aalloc<float>(a, 6 * field_elems(p)));
        a->ck_psi.push_back(p.npml > 0 ? aalloc<float>(a, psi_total(p)) : nullptr);
        a->ck_par.push_back(0);
    }
    check(hipMemcpyAsync(a->ck_f[q], p.fbase[c->parity], field_bytes(p), hipMemcpyDeviceToDevice,
                         c->stream), "checkpoint");
    if (psi_bytes(p))
        check(hipMemcpyAsync(a->ck_psi[q], p.pbase[c->parity], psi_bytes(p),
                             hipMemcpyDeviceToDevice, c->stream), "checkpoint");
    a->ck_par[q] = c->parity;
}

void restore_checkpoint(fdtd_adjoint* a, int q) {
    fdtd_ctx* c = a->c;
    const Problem& p = c->p;
    const int par = a->ck_par[q];
    check(hipMemcpyAsync(p.fbase[par], a->ck_f[q], field_bytes(p), hipMemcpyDeviceToDevice,
                         c->stream), "restore");
    if (psi_bytes(p))
        check(hipMemcpyAsync(p.pbase[par], a->ck_psi[q], psi_bytes(p), hipMemcpyDeviceToDevice,
                             c->stream), "restore");
    c->parity = par;
    c->step = (long long)q * a->every;
    c->energy_valid = false;
}

// Forward steps n0 .. n1-1 from the restored checkpoint with the plane
// accumulation off, recording E_y^{n+1} of the plane for n >= rec_begin.
void recompute(fdtd_adjoint* a, long long n0, long long n1, long long rec_begin) {
    fdtd_ctx* c = a->c;
    for (long long n = n0; n < n1; ++n) {
        Problem q = c->p;
        q.diag_mask = 0;
        q.plane = a->plane;
        q.rec = n >= rec_begin ? a->rec : nullptr;
        q.rec_begin = rec_begin;
        check(launch_step(c, q, n, c->parity, nullptr), "recompute launch");
        c->parity ^= 1;
        c->step = n + 1;
        a->recompute_steps += 1;
    }
}

void upload_slots(fdtd_adjoint* a) {
    const Antenna& ant = a->c->ant;
    const int ns = (int)ant.slot_i.size();
    if (ns > a->nslots || !a->slot_i) {
        afree(a, a->slot_i);
        afree(a, a->slot_j);
        afree(a, a->G);
        a->slot_i = aalloc<int>(a, ns);
        a->slot_j = aalloc<int>(a, ns);
        a->G = aalloc<double2>(a, (size_t)ns * 6);
    }
    a->nslots = ns;
    if (ns > 0) {
        check(hipMemcpyAsync(a->slot_i, ant.slot_i.data(), ns * sizeof(int), hipMemcpyHostToDevice,
                             a->c->stream), "copy slots");
        check(hipMemcpyAsync(a->slot_j, ant.slot_j.data(), ns * sizeof(int), hipMemcpyHostToDevice,
                             a->c->stream), "copy slots");
    }
    check(hipStreamSynchronize(a->c->stream), "sync");
}

// T(t) = f(t) e^{-iω(t - T0)} at t = steps·Δt, rounded to float as in the
// forward time tables (the gradient is that of the computed forward run).
float2 time_value(const fdtd_ctx* c, double steps) {
    double re, im;
    time_factor(c->ant, steps * c->g.courant, &re, &im);
    return make_float2((float)re, (float)im);
}

// Host copy of one λ array (fields and ψ of the current parity), same host
// layouts as fdtd_get_state.
void state_copy(fdtd_adjoint* a, int which, float* host, int64_t n, bool to_host,
                const Problem& p) {
    need(which >= FDTD_EX && which <= FDTD_PSI_HZY, "unknown state array");
    size_t ne;
    const bool xslab = which == FDTD_PSI_EYX || which == FDTD_PSI_EZX || which == FDTD_PSI_HYX ||
                       which == FDTD_PSI_HZX;
    if (which <= FDTD_HZ) ne = (size_t)p.nz * p.ny * p.nx;
    else if (p.npml == 0) ne = 0;
    else if (xslab) ne = (size_t)p.nz * p.ny * 2 * p.npml;
    else ne = (size_t)p.nz * 2 * p.npml * p.nx;
    need(ne > 0, "array not present (no CPML)");
    need(host && n == (int64_t)ne, "element count mismatch");
    hipStream_t s = a->c->stream;
    const size_t w = p.nx * sizeof(float), pb = p.pitch * sizeof(float);
    if (which <= FDTD_HZ) {
        float* d = p.fbase[a->lam_par] + which * p.fstride;
        if (to_host)
            check(hipMemcpy2DAsync(host, w, d, pb, w, (size_t)p.nz * p.ny, hipMemcpyDeviceToHost, s), "copy");
        else
            check(hipMemcpy2DAsync(d, pb, host, w, w, (size_t)p.nz * p.ny, hipMemcpyHostToDevice, s), "copy");
    } else {
        float* d = p.pbase[a->lam_par] + psi_offset(p, which - FDTD_PSI_EXY);
        if (xslab) {
            check(hipMemcpyAsync(to_host ? (void*)host : (void*)d, to_host ? (const void*)d : (const void*)host,
                                 ne * sizeof(float), to_host ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice, s), "copy");
        } else if (to_host) {
            check(hipMemcpy2DAsync(host, w, d, pb, w, (size_t)p.nz * 2 * p.npml, hipMemcpyDeviceToHost, s), "copy");
        } else {
            check(hipMemcpy2DAsync(d, pb, host, w, w, (size_t)p.nz * 2 * p.npml, hipMemcpyHostToDevice, s), "copy");
        }
    }
    check(hipStreamSynchronize(s), "sync");
}

}  // namespace

extern "C" {

int fdtd_adjoint_create(fdtd_ctx* fwd, int32_t checkpoint_every, fdtd_adjoint** out) {
    if (!out) return FDTD_EINVAL;
    *out = nullptr;
    if (!fwd || checkpoint_every < 1) {
        g_adj_create_error = "need a forward context and checkpoint_every >= 1";
        return FDTD_EINVAL;
    }
    if (fwd->batch_owned) {
        g_adj_create_error = "the forward context is stepped by a batch";
        return FDTD_ESTATE;
    }
    fdtd_adjoint* a = new (std::nothrow) fdtd_adjoint();
    if (!a) return FDTD_ENOMEM;
    a->c = fwd;
    a->every = checkpoint_every;
    try {
        fwd->adjoints.push_back(a);
    } catch (...) {
        delete a;
        return FDTD_ENOMEM;
    }
    int rc = aguard(a, [&] {
        const Problem& f = fwd->p;
        Problem& l = a->lam;
        l = f;
        for (int par = 0; par < 2; ++par) l.fbase[par] = aalloc<float>(a, 6 * field_elems(f));
        for (int par = 0; par < 2; ++par)
            l.pbase[par] = f.npml > 0 ? aalloc<float>(a, psi_total(f)) : nullptr;
        l.fl = nullptr;
        l.rec = nullptr;
        l.diag_mask = 0;
        a->rec = aalloc<float>(a, (size_t)checkpoint_every * f.nx * f.ny);
        a->g_dev = aalloc<float>(a, (size_t)f.nx * f.ny);
        clear_lambda(a);
        check(hipStreamSynchronize(fwd->stream), "sync");
    });
    if (rc != FDTD_OK) {
        g_adj_create_error = a->err;
        fdtd_adjoint_destroy(a);
        return rc;
    }
    *out = a;
    return FDTD_OK;
}

int fdtd_adjoint_destroy(fdtd_adjoint* a) {
    if (!a) return FDTD_OK;
    if (a->c) {
        (void)hipStreamSynchronize(a->c->stream);
        auto& v = a->c->adjoints;
        v.erase(std::remove(v.begin(), v.end(), a), v.end());
    }
    // (a detached adjoint: fdtd_destroy synchronised the stream its work ran on)
    for (const auto& q : a->allocs) (void)hipFree(q.first);
    delete a;
    return FDTD_OK;
}

const char* fdtd_adjoint_last_error(const fdtd_adjoint* a) {
    return a ? a->err.c_str() : g_adj_create_error.c_str();
}

int fdtd_adjoint_forward(fdtd_adjoint* a, int64_t nsteps, int32_t plane, int64_t window_begin) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        fdtd_ctx* c = a->c;
        need(c->has_inj, "the forward context has no injector", FDTD_ESTATE);
        need(nsteps >= 1, "nsteps must be >= 1");
        need(window_begin >= 0 && window_begin < nsteps, "window must lie inside the run");
        need(plane >= 0 && plane < c->p.nz, "plane out of range");
        a->have_forward = false;
        int rc = fdtd_reset(c);
        if (rc != FDTD_OK) throw Fail{rc, c->err};
        rc = fdtd_set_diagnostics(c, plane, window_begin, FDTD_DIAG_EY2);
        if (rc != FDTD_OK) throw Fail{rc, c->err};
        a->nsteps = nsteps;
        a->wbegin = window_begin;
        a->plane = plane;
        const int nck = (int)((nsteps + a->every - 1) / a->every);
        for (int q = 0; q < nck; ++q) {
            save_checkpoint(a, q);
            const long long m = std::min<long long>(a->every, nsteps - (long long)q * a->every);
            rc = fdtd_step(c, m);
            if (rc != FDTD_OK) throw Fail{rc, c->err};
        }
        upload_slots(a);
        a->inj_version = c->inj_version;
        a->have_forward = true;
        ++a->runs;
    });
}

int fdtd_adjoint_backward(fdtd_adjoint* a, const float* dl_dI, int64_t n, int32_t n_sectors,
                          double* grad_amp, double* grad_phase) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        fdtd_ctx* c = a->c;
        need(a->have_forward, "run fdtd_adjoint_forward first", FDTD_ESTATE);
        need(c->has_inj, "the forward context has no injector", FDTD_ESTATE);
        need(a->inj_version == c->inj_version,
             "the antenna or its sector weights changed since fdtd_adjoint_forward; run it again",
             FDTD_ESTATE);
        const Problem& p = c->p;
        need(dl_dI && n == (int64_t)p.nx * p.ny, "dL/dI must hold ny*nx values");
        need(n_sectors == c->ant.n_sectors && n_sectors > 0 && grad_amp && grad_phase,
             "sector count mismatch");
        hipStream_t s = c->stream;
        ensure_time_tables(c, a->nsteps + 1);
        check(hipMemcpyAsync(a->g_dev, dl_dI, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s),
              "copy dL/dI");
        clear_lambda(a);
        sync_lambda_tables(a);
        if (a->nslots > 0)
            check(hipMemsetAsync(a->G, 0, (size_t)a->nslots * 6 * sizeof(double2), s), "clear G");
        const float coef = (float)(2.0 / (double)(a->nsteps - a->wbegin));
        a->recompute_steps = 0;
        const int nck = (int)((a->nsteps + a->every - 1) / a->every);
        for (int q = nck - 1; q >= 0; --q) {
            const long long n0 = (long long)q * a->every;
            const long long n1 = std::min<long long>(n0 + a->every, a->nsteps);
            const long long rb = std::max(n0, a->wbegin);
            if (n1 > a->wbegin) {
                restore_checkpoint(a, q);
                recompute(a, n0, n1, rb);
            }
            for (long long m = n1 - 1; m >= n0; --m) {
                if (m >= a->wbegin)
                    check(launch_adjoint_inject(a->lam, a->lam_par, a->g_dev,
                                                a->rec + (size_t)(m - rb) * p.nx * p.ny, coef, s),
                          "inject");
                reverse_step(a, true, m);
            }
        }
        // sector gradients from the per-point correlations (host, double)
        std::vector<double2> G((size_t)a->nslots * 6);
        if (a->nslots > 0)
            check(hipMemcpyAsync(G.data(), a->G, G.size() * sizeof(double2), hipMemcpyDeviceToHost,
                                 s), "copy G");
        check(hipStreamSynchronize(s), "sync");
        const Antenna& ant = c->ant;
        std::fill(grad_amp, grad_amp + n_sectors, 0.0);
        std::fill(grad_phase, grad_phase + n_sectors, 0.0);
        for (int q = 0; q < a->nslots * 6; ++q) {
            if (!ant.member[q]) continue;
            const int sec = ant.sector[q];
            const std::complex<double> base(ant.base_re[q], ant.base_im[q]);
            const std::complex<double> g(G[q].x, G[q].y);
            const std::complex<double> rot = std::polar(1.0, ant.sec_phase[sec]);
            grad_amp[sec] += std::real(rot * base * g);
            grad_phase[sec] -= std::imag(ant.sec_amp[sec] * rot * base * g);
        }
    });
}

int fdtd_adjoint_source_correlation(fdtd_adjoint* a, double* host, int64_t n) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        need(a->G != nullptr, "no backward run yet", FDTD_ESTATE);
        need(host && n == (int64_t)a->nslots * 12, "need 12 doubles per antenna column");
        check(hipMemcpyAsync(host, a->G, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                             a->c->stream), "copy G");
        check(hipStreamSynchronize(a->c->stream), "sync");
    });
}

int fdtd_adjoint_transpose(fdtd_adjoint* a, int64_t nsteps) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        need(nsteps >= 0, "nsteps must be >= 0");
        sync_lambda_tables(a);
        for (int64_t q = 0; q < nsteps; ++q) transposed_step(a);
    });
}

int fdtd_adjoint_get_state(fdtd_adjoint* a, int32_t which, float* host, int64_t n) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        const Problem& p = a->lam;
        state_copy(a, which, host, n, true, p);
    });
}

int fdtd_adjoint_set_state(fdtd_adjoint* a, int32_t which, const float* host, int64_t n) {
    if (!a) return FDTD_EINVAL;
    return aguard(a, [&] {
        attached(a);
        const Problem& p = a->lam;
        state_copy(a, which, const_cast<float*>(host), n, false, p);
    });
}

int fdtd_adjoint_get_info(const fdtd_adjoint* a, fdtd_adjoint_info* out) {
    if (!a || !out) return FDTD_EINVAL;
    fdtd_adjoint_info r{};
    r.checkpoint_every = a->every;
    r.checkpoints = (int32_t)a->ck_f.size();
    r.antenna_columns = a->nslots;
    r.forward_steps = a->nsteps;
    r.recompute_steps = a->recompute_steps;
    r.device_bytes = a->device_bytes;
    r.forward_runs = a->runs;
    *out = r;
    return FDTD_OK;
}

}  // extern "C"
