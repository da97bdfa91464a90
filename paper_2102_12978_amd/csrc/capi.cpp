// C ABI of the Bessel-antenna FDTD solver: context life cycle, device
// buffers, antenna tables, the step loop and read-backs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"

using namespace bfdtd;


namespace {

thread_local std::string g_create_error;
const char* kVersion = "besselfdtd 0.1 (gfx950)";

size_t state_elems(const fdtd_ctx* c, int which) {
    const Problem& p = c->p;
    if (which >= FDTD_EX && which <= FDTD_HZ) return (size_t)p.nz * p.ny * p.nx;
    if (p.npml == 0) return 0;
    switch (which) {
        case FDTD_PSI_EYX: case FDTD_PSI_EZX: case FDTD_PSI_HYX: case FDTD_PSI_HZX:
            return (size_t)p.nz * p.ny * 2 * p.npml;
        default:
            return (size_t)p.nz * 2 * p.npml * p.nx;
    }
}

bool psi_is_x(int which) {
    return which == FDTD_PSI_EYX || which == FDTD_PSI_EZX || which == FDTD_PSI_HYX ||
           which == FDTD_PSI_HZX;
}

void launch_one(fdtd_ctx* c, long long n) {
    Problem q = c->p;
    const bool in_window = c->plane >= 0 && n >= c->wbegin;
    q.diag_mask = in_window ? (int)(c->mask & 7u) : 0;
    q.plane = c->plane;
    double* ep = (c->mask & FDTD_DIAG_ENERGY) ? c->epart : nullptr;
    check(launch_step(c, q, n, c->parity, ep), "step launch");
    if (ep) {
        if (c->timer) c->timer->mark("energy_reduce");
        check(launch_energy_reduce(c->epart, partial_count(c), c->energy_dev, c->stream),
              "energy reduce");
        if (c->timer) c->timer->mark(nullptr);
        c->energy_valid = true;
    }
    if (q.diag_mask) c->count += 1;
    c->parity ^= 1;
    c->step += 1;
    // bound the number of outstanding timing events
    if (c->timer && c->timer->open_.size() > 4096) c->timer->collect();
}

}  // namespace

extern "C" {

const char* fdtd_version(void) { return kVersion; }

int fdtd_fit_periodic_z(double wavelength, double theta, double dx, int32_t nz_hint, int32_t* nz,
                        double* dz) {
    if (!nz || !dz) return FDTD_EINVAL;
    if (!(wavelength > 0) || !(dx > 0) || nz_hint < 1 || !(theta > 0) ||
        !(theta < 1.5707963267948966))
        return FDTD_EINVAL;
    double lam_z = wavelength / std::cos(theta);
    double p = std::max(1.0, std::floor(nz_hint * dx / lam_z + 0.5));
    double n = std::max(1.0, std::floor(p * lam_z / dx + 0.5));
    if (n > 2147483647.0) return FDTD_EINVAL;
    *nz = (int32_t)n;
    *dz = p * lam_z / n;
    return FDTD_OK;
}

int fdtd_antenna_points(const fdtd_grid* grid, const fdtd_injector* inj, int32_t* out,
                        int64_t cap, int64_t* count) {
    if (!grid || !inj || !count || cap < 0 || (cap > 0 && !out)) return FDTD_EINVAL;
    try {
        if (!validate_grid(*grid).empty()) return FDTD_EINVAL;
        Antenna a;
        if (!build_antenna(*grid, 0, grid->dy / grid->dx, grid->dz / grid->dx, *inj, &a).empty())
            return FDTD_EINVAL;
        int64_t n = 0;
        for (size_t s = 0; s < a.slot_i.size(); ++s)
            for (int c = 0; c < 6; ++c) {
                if (!a.member[s * 6 + c]) continue;
                if (n < cap) {
                    int32_t* q = out + 4 * n;
                    q[0] = c;
                    q[1] = a.slot_i[s];
                    q[2] = a.slot_j[s];
                    q[3] = a.n_sectors > 0 ? a.sector[s * 6 + c] : -1;
                }
                ++n;
            }
        *count = n;
        return n <= cap ? FDTD_OK : FDTD_EINVAL;
    } catch (...) {
        return FDTD_ENOMEM;
    }
}

const char* fdtd_last_error(const fdtd_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

namespace {

// fdtd_create / fdtd_create_ext: ext is NULL (the library allocates the two
// field parities) or the caller's two parity buffers.
int create_impl(const fdtd_grid* grid, float* const* ext, fdtd_ctx** out) {
    if (!out) return FDTD_EINVAL;
    *out = nullptr;
    if (!grid) {
        g_create_error = "grid is NULL";
        return FDTD_EINVAL;
    }
    std::string v = validate_grid(*grid);
    if (!v.empty()) {
        g_create_error = v;
        return FDTD_EINVAL;
    }
    fdtd_ctx* c = new (std::nothrow) fdtd_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return FDTD_ENOMEM;
    }
    int rc = guarded(c, [&] {
        int ndev = 0;
        check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        need(ndev > 0, "no HIP device", FDTD_EDEVICE);
        check(hipGetDevice(&c->device), "hipGetDevice");
        c->g = *grid;
        c->stream = (hipStream_t)grid->stream;
        c->ry = grid->dy / grid->dx;
        c->rz = grid->dz / grid->dx;
        c->kernel = grid->kernel == FDTD_KERNEL_SPLIT ? FDTD_KERNEL_SPLIT : FDTD_KERNEL_FUSED;
        Problem& p = c->p;
        p.nx = grid->nx;
        p.ny = grid->ny;
        p.nz = grid->nz;
        p.pitch = (grid->nx + 63) / 64 * 64;   // 256-byte rows
        p.npml = grid->bc_xy == FDTD_BC_CPML ? grid->cpml_cells : 0;
        p.periodic = grid->bc_xy == FDTD_BC_PERIODIC;
        p.plane = -1;
        p.sx = (float)grid->courant;
        p.sy = (float)(grid->courant / c->ry);
        p.sz = (float)(grid->courant / c->rz);
        p.fstride = (long long)field_elems(p);
        need((size_t)p.ny * p.pitch * sizeof(float) < (1ull << 31),
             "one z plane of a field component must stay below 2 GiB (32-bit offsets)");
        if (p.npml > 0) {
            p.psx = (long long)psix_elems(p);
            p.psy = (long long)psiy_elems(p);
        }
        if (ext) {
            // Reject what the kernels could not use before anything runs on
            // it: a buffer outside device memory of this device, misaligned,
            // running past its allocation, or overlapping the other one.
            const size_t bytes = 6 * field_elems(p) * sizeof(float);
            for (int par = 0; par < 2; ++par) {
                float* f = ext[par];
                need(f != nullptr, "dev_fields[] must not be NULL");
                need(((uintptr_t)f & 255u) == 0, "dev_fields[] must be 256-byte aligned");
                hipPointerAttribute_t at{};
                const bool dev = hipPointerGetAttributes(&at, f) == hipSuccess &&
                                 at.type == hipMemoryTypeDevice && at.device == c->device;
                hipDeviceptr_t base = nullptr;
                size_t size = 0;
                const bool inside =
                    dev && hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)f) == hipSuccess &&
                    (const char*)f + bytes <= (const char*)base + size;
                (void)hipGetLastError();   // a failed query leaves no error behind
                need(dev, "dev_fields[] must be device memory of the current device");
                need(inside, "dev_fields[] buffer ends before the field layout does");
            }
            const char *a0 = (const char*)ext[0], *a1 = (const char*)ext[1];
            need(a0 + bytes <= a1 || a1 + bytes <= a0, "dev_fields[0] and [1] overlap");
        }
        for (int par = 0; par < 2; ++par) {
            if (ext) {
                p.fbase[par] = ext[par];
                check(hipMemsetAsync(ext[par], 0, 6 * field_elems(p) * sizeof(float), c->stream),
                      "clear fields");
            } else {
                p.fbase[par] = dalloc<float>(c, 6 * field_elems(p));
            }
            p.pbase[par] = p.npml > 0 ? dalloc<float>(c, psi_total(p)) : nullptr;
        }
        std::vector<float> tx[6], ty[6];
        cpml_axis_tables(p.nx, p.npml, 1.0, *grid, grid->courant, tx);
        cpml_axis_tables(p.ny, p.npml, c->ry, *grid, grid->courant, ty);
        std::vector<float> tab;
        for (int t = 0; t < 6; ++t) tab.insert(tab.end(), tx[t].begin(), tx[t].end());
        for (int t = 0; t < 6; ++t) tab.insert(tab.end(), ty[t].begin(), ty[t].end());
        float* tabs = dalloc<float>(c, tab.size());
        check(hipMemcpyAsync(tabs, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice,
                             c->stream), "copy cpml");
        p.ctab = tabs;
        c->fl = dalloc<double>(c, 3 * (size_t)p.nx * p.ny);
        p.fl = c->fl;
        c->energy_dev = dalloc<double>(c, 1);
        int cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
        c->zchunk = fused_default_zchunk(p, c->rows, c->xalign, cus);
        ensure_partials(c);
        check(hipStreamSynchronize(c->stream), "sync");
    });
    if (rc != FDTD_OK) {
        g_create_error = c->err;
        fdtd_destroy(c);
        return rc;
    }
    *out = c;
    return FDTD_OK;
}

}  // namespace

int fdtd_create(const fdtd_grid* grid, fdtd_ctx** out) { return create_impl(grid, nullptr, out); }

int fdtd_create_ext(const fdtd_grid* grid, float* const dev_fields[2], fdtd_ctx** out) {
    if (!dev_fields) {
        if (out) *out = nullptr;
        g_create_error = "dev_fields is NULL";
        return FDTD_EINVAL;
    }
    return create_impl(grid, dev_fields, out);
}

int fdtd_field_layout(const fdtd_grid* grid, int32_t* pitch, int64_t* parity_floats) {
    if (!grid || !pitch || !parity_floats) return FDTD_EINVAL;
    if (!validate_grid(*grid).empty()) return FDTD_EINVAL;
    const int64_t pt = ((int64_t)grid->nx + 63) / 64 * 64;
    *pitch = (int32_t)pt;
    *parity_floats = 6 * (int64_t)grid->nz * grid->ny * pt;
    return FDTD_OK;
}

int fdtd_current_fields(const fdtd_ctx* c, float** dev_ptr) {
    if (!c || !dev_ptr) return FDTD_EINVAL;
    *dev_ptr = c->p.fbase[c->parity];
    return FDTD_OK;
}

int fdtd_destroy(fdtd_ctx* ctx) {
    if (!ctx) return FDTD_OK;
    if (ctx->batch_owned) {
        ctx->err = "instance is owned by its batch";
        return FDTD_ESTATE;
    }
    if (!ctx->allocs.empty()) (void)hipStreamSynchronize(ctx->stream);
    for (fdtd_adjoint* a : ctx->adjoints) detach_adjoint(a);
    destroy_side_streams(ctx);
    delete ctx->timer;
    for (const auto& a : ctx->allocs) (void)hipFree(a.first);
    delete ctx;
    return FDTD_OK;
}

int fdtd_set_injector(fdtd_ctx* c, const fdtd_injector* inj) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        if (!inj) {
            check(hipStreamSynchronize(c->stream), "sync");
            dfree(c, c->colmap); dfree(c, c->amp); dfree(c, c->zph);
            dfree(c, c->tE); dfree(c, c->tH);
            c->colmap = nullptr; c->amp = nullptr; c->zph = nullptr;
            c->tE = c->tH = nullptr;
            c->t_cap = 0;
            c->has_inj = false;
            c->p.colmap = nullptr; c->p.amp = nullptr; c->p.zph = nullptr;
            c->p.tE = c->p.tH = nullptr;
            c->p.n_slots = 0;
            ++c->inj_version;
            return;
        }
        Antenna a;
        std::string msg = build_antenna(c->g, c->p.pitch, c->ry, c->rz, *inj, &a);
        need(msg.empty(), msg);
        check(hipStreamSynchronize(c->stream), "sync");
        dfree(c, c->colmap); dfree(c, c->amp); dfree(c, c->zph);
        dfree(c, c->tE); dfree(c, c->tH);
        c->tE = c->tH = nullptr;
        c->t_cap = 0;
        c->ant = std::move(a);
        const Problem& p = c->p;
        const int ns = (int)c->ant.slot_i.size();
        std::vector<int> map((size_t)p.nx * p.ny, -1);
        for (int s = 0; s < ns; ++s) map[(size_t)c->ant.slot_j[s] * p.nx + c->ant.slot_i[s]] = s;
        std::vector<float> amp;
        weighted_amplitudes(c->ant, &amp);
        std::vector<float2> zph(2 * (size_t)p.nz);
        for (int k = 0; k < p.nz; ++k) {
            double z0 = c->ant.beta * k * c->rz, z1 = c->ant.beta * (k + 0.5) * c->rz;
            zph[2 * k] = make_float2((float)std::cos(z0), (float)std::sin(z0));
            zph[2 * k + 1] = make_float2((float)std::cos(z1), (float)std::sin(z1));
        }
        c->colmap = dalloc<int>(c, map.size());
        c->amp = dalloc<float2>(c, std::max<size_t>(1, (size_t)ns * 6));
        c->zph = dalloc<float2>(c, zph.size());
        check(hipMemcpyAsync(c->colmap, map.data(), map.size() * sizeof(int),
                             hipMemcpyHostToDevice, c->stream), "copy map");
        if (ns > 0)
            check(hipMemcpyAsync(c->amp, amp.data(), amp.size() * sizeof(float),
                                 hipMemcpyHostToDevice, c->stream), "copy amp");
        check(hipMemcpyAsync(c->zph, zph.data(), zph.size() * sizeof(float2),
                             hipMemcpyHostToDevice, c->stream), "copy zph");
        c->p.colmap = c->colmap;
        c->p.amp = c->amp;
        c->p.zph = c->zph;
        c->p.n_slots = ns;
        c->has_inj = true;
        ++c->inj_version;
        ensure_time_tables(c, c->step + 1024);
    });
}

int fdtd_set_sector_weights(fdtd_ctx* c, int32_t n, const double* amp, const double* phase) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(c->has_inj, "no injector", FDTD_ESTATE);
        need(n == c->ant.n_sectors && n > 0 && amp && phase, "sector count mismatch");
        for (int s = 0; s < n; ++s) {
            c->ant.sec_amp[s] = amp[s];
            c->ant.sec_phase[s] = phase[s];
        }
        ++c->inj_version;
        std::vector<float> w;
        weighted_amplitudes(c->ant, &w);
        if (!w.empty())
            check(hipMemcpyAsync(c->amp, w.data(), w.size() * sizeof(float),
                                 hipMemcpyHostToDevice, c->stream), "copy amp");
        check(hipStreamSynchronize(c->stream), "sync");
    });
}

int fdtd_set_diagnostics(fdtd_ctx* c, int32_t k_plane, int64_t window_begin_step, uint32_t mask) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(k_plane >= -1 && k_plane < c->p.nz, "plane out of range");
        need(window_begin_step >= 0, "window begin must be >= 0");
        need((mask & ~15u) == 0, "unknown diagnostics bits");
        need(k_plane >= 0 || (mask & 7u) == 0, "plane quantities need a plane");
        c->plane = k_plane;
        c->wbegin = window_begin_step;
        c->mask = mask;
        c->count = 0;
        c->energy_valid = false;
        check(hipMemsetAsync(c->fl, 0, 3 * (size_t)c->p.nx * c->p.ny * sizeof(double), c->stream),
              "clear fluence");
        ensure_partials(c);
    });
}

int fdtd_step(fdtd_ctx* c, int64_t nsteps) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(nsteps >= 0, "nsteps must be >= 0");
        ensure_time_tables(c, c->step + nsteps);
        ensure_partials(c);
        const bool pairs = two_step_on(c), triples = three_step_on(c);
        for (int64_t s = 0; s < nsteps;) {
            if (triples && nsteps - s >= 3) {
                launch_triple(c, c->step);
                s += 3;
            } else if (pairs && nsteps - s >= 2) {
                launch_pair(c, c->step);
                s += 2;
            } else {
                launch_one(c, c->step);
                s += 1;
            }
        }
    });
}

int fdtd_fluence(fdtd_ctx* c, uint32_t quantity, float* host_out, int64_t n) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        int ch = quantity == FDTD_DIAG_EX2 ? 0 : quantity == FDTD_DIAG_EY2 ? 1
               : quantity == FDTD_DIAG_EZ2 ? 2 : -1;
        need(ch >= 0, "quantity must be one of FDTD_DIAG_EX2/EY2/EZ2");
        const size_t np = (size_t)c->p.nx * c->p.ny;
        need(host_out && n >= (int64_t)np, "output buffer too small");
        std::vector<double> h(np);
        check(hipMemcpyAsync(h.data(), c->fl + ch * np, np * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream), "copy fluence");
        check(hipStreamSynchronize(c->stream), "sync");
        const double inv = c->count > 0 ? 1.0 / (double)c->count : 0.0;
        bool finite = true;
        for (size_t q = 0; q < np; ++q) {
            host_out[q] = (float)(h[q] * inv);
            finite = finite && std::isfinite(h[q]);
        }
        need(finite, "fluence is not finite (the run has diverged)", FDTD_EUNSTABLE);
    });
}

int fdtd_fluence_count(const fdtd_ctx* c, int64_t* count) {
    if (!c || !count) return FDTD_EINVAL;
    *count = c->count;
    return FDTD_OK;
}

int fdtd_energy(fdtd_ctx* c, double* out) {
    if (!c || !out) return FDTD_EINVAL;
    int rc = guarded(c, [&] {
        need(c->energy_valid, "energy diagnostics not enabled or no step taken", FDTD_ESTATE);
        check(hipMemcpyAsync(out, c->energy_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream),
              "copy energy");
        check(hipStreamSynchronize(c->stream), "sync");
    });
    if (rc == FDTD_OK && !std::isfinite(*out)) {
        c->err = "energy is not finite";
        return FDTD_EUNSTABLE;
    }
    return rc;
}

int fdtd_get_state(fdtd_ctx* c, int32_t which, float* host, int64_t n) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(which >= FDTD_EX && which <= FDTD_PSI_HZY, "unknown state array");
        size_t ne = state_elems(c, which);
        need(ne > 0, "array not present (no CPML)");
        need(host && n == (int64_t)ne, "element count mismatch");
        const Problem& p = c->p;
        if (which <= FDTD_HZ) {
            check(hipMemcpy2DAsync(host, p.nx * sizeof(float), p.fbase[c->parity] + which * p.fstride,
                                   p.pitch * sizeof(float), p.nx * sizeof(float),
                                   (size_t)p.nz * p.ny, hipMemcpyDeviceToHost, c->stream),
                  "copy field");
        } else if (psi_is_x(which)) {
            check(hipMemcpyAsync(host, p.pbase[c->parity] + psi_offset(p, which - FDTD_PSI_EXY),
                                 ne * sizeof(float),
                                 hipMemcpyDeviceToHost, c->stream), "copy psi");
        } else {
            check(hipMemcpy2DAsync(host, p.nx * sizeof(float),
                                   p.pbase[c->parity] + psi_offset(p, which - FDTD_PSI_EXY),
                                   p.pitch * sizeof(float), p.nx * sizeof(float),
                                   (size_t)p.nz * 2 * p.npml, hipMemcpyDeviceToHost, c->stream),
                  "copy psi");
        }
        check(hipStreamSynchronize(c->stream), "sync");
    });
}

int fdtd_set_state(fdtd_ctx* c, int32_t which, const float* host, int64_t n) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(which >= FDTD_EX && which <= FDTD_PSI_HZY, "unknown state array");
        size_t ne = state_elems(c, which);
        need(ne > 0, "array not present (no CPML)");
        need(host && n == (int64_t)ne, "element count mismatch");
        const Problem& p = c->p;
        if (which <= FDTD_HZ) {
            check(hipMemcpy2DAsync(p.fbase[c->parity] + which * p.fstride, p.pitch * sizeof(float), host,
                                   p.nx * sizeof(float), p.nx * sizeof(float), (size_t)p.nz * p.ny,
                                   hipMemcpyHostToDevice, c->stream), "copy field");
        } else if (psi_is_x(which)) {
            check(hipMemcpyAsync(p.pbase[c->parity] + psi_offset(p, which - FDTD_PSI_EXY), host,
                                 ne * sizeof(float),
                                 hipMemcpyHostToDevice, c->stream), "copy psi");
        } else {
            check(hipMemcpy2DAsync(p.pbase[c->parity] + psi_offset(p, which - FDTD_PSI_EXY),
                                   p.pitch * sizeof(float),
                                   host, p.nx * sizeof(float), p.nx * sizeof(float),
                                   (size_t)p.nz * 2 * p.npml, hipMemcpyHostToDevice, c->stream),
                  "copy psi");
        }
        check(hipStreamSynchronize(c->stream), "sync");
        c->energy_valid = false;
    });
}

int fdtd_reset(fdtd_ctx* c) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        const Problem& p = c->p;
        for (int par = 0; par < 2; ++par) {
            check(hipMemsetAsync(p.fbase[par], 0, 6 * field_elems(p) * sizeof(float), c->stream),
                  "clear");
            if (p.npml > 0)
                check(hipMemsetAsync(p.pbase[par], 0, psi_total(p) * sizeof(float), c->stream),
                      "clear");
        }
        check(hipMemsetAsync(c->fl, 0, 3 * (size_t)p.nx * p.ny * sizeof(double), c->stream),
              "clear");
        check(hipStreamSynchronize(c->stream), "sync");
        c->step = 0;
        c->parity = 0;
        c->count = 0;
        c->energy_valid = false;
    });
}

int fdtd_get_info(const fdtd_ctx* c, fdtd_info* out) {
    if (!c || !out) return FDTD_EINVAL;
    std::memset(out, 0, sizeof *out);
    out->nx = c->p.nx;
    out->ny = c->p.ny;
    out->nz = c->p.nz;
    out->pitch = c->p.pitch;
    out->sx = c->g.courant;
    out->sy = c->g.courant / c->ry;
    out->sz = c->g.courant / c->rz;
    if (c->has_inj) {
        out->k = c->ant.k;
        out->beta = c->ant.beta;
        out->kr = c->ant.kr;
        out->omega = c->ant.omega;
        for (int q = 0; q < 6; ++q) out->n_source[q] = c->ant.n_source[q];
        out->n_slots = (int32_t)c->ant.slot_i.size();
    }
    out->kernel = c->kernel;
    out->tile_rows = c->rows;
    out->tile_zchunk = c->zchunk;
    out->frame = c->frame;
    out->xalign = c->xalign;
    out->frame_rows = c->frame_rows;
    out->time_block = c->time_block;
    out->tb_rows = c->tb_rows;
    out->tb_zchunk = c->tb_zchunk;
    out->step = c->step;
    out->device_bytes = c->device_bytes;
    if (three_step_on(c)) {
        out->interior_cells = step3_interior_cells(c->p, c->tb_rows);
    } else if (two_step_on(c)) {
        out->interior_cells = step2_interior_cells(c->p, c->tb_rows);
    } else {
        const Frame fr = interior_of(c);
        out->interior_cells = (long long)(fr.x1 - fr.x0) * (fr.y1 - fr.y0) * c->p.nz;
    }
    return FDTD_OK;
}

int fdtd_analytic_ey2(fdtd_ctx* c, float* host_out, int64_t n) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(c->has_inj, "no injector", FDTD_ESTATE);
        need(c->ant.polarization == FDTD_POL_X_TE,
             "the analytic E_y intensity is that of the Pi_x TE beam", FDTD_ESTATE);
        const Problem& p = c->p;
        need(host_out && n >= (int64_t)p.nx * p.ny, "output buffer too small");
        const Antenna& a = c->ant;
        const double amp = 0.5 * a.e0 * a.e0 * std::cos(a.theta) * std::cos(a.theta);
        for (int j = 0; j < p.ny; ++j) {
            for (int i = 0; i < p.nx; ++i) {
                double r = std::hypot(i - a.ax, (j + 0.5) * c->ry - a.ay);
                double v = std::cyl_bessel_j((double)a.order, a.kr * r);
                host_out[(size_t)j * p.nx + i] = (float)(amp * v * v);
            }
        }
    });
}

int fdtd_set_tile(fdtd_ctx* c, int32_t rows, int32_t zchunk) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(rows == 4 || rows == 8, "rows must be 4 or 8");
        need(zchunk >= 0 && zchunk <= c->p.nz, "zchunk out of range");
        c->rows = rows;
        c->zchunk = zchunk;
        ensure_partials(c);
    });
}

int fdtd_set_time_block(fdtd_ctx* c, int32_t steps, int32_t rows, int32_t zchunk) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(steps >= 1 && steps <= 3, "steps must be 1, 2 or 3");
        need(rows == 2 || rows == 4, "rows must be 2 or 4");
        need(zchunk >= 0 && zchunk <= c->p.nz, "zchunk out of range");
        c->time_block = steps;
        c->tb_rows = rows;
        c->tb_zchunk = zchunk;
    });
}

int fdtd_set_concurrency(fdtd_ctx* c, int32_t on) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(on == 0 || on == 1, "on must be 0 or 1");
        c->concurrent = on != 0;
    });
}

int fdtd_set_frame(fdtd_ctx* c, int32_t kind, int32_t xalign, int32_t rows) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(kind == FDTD_FRAME_SPLIT || kind == FDTD_FRAME_FUSED,
             "kind must be FDTD_FRAME_SPLIT or FDTD_FRAME_FUSED");
        need(xalign == 32 || xalign == 64, "xalign must be 32 or 64");
        need(rows == 2 || rows == 4, "rows must be 2 or 4");
        c->frame = kind;
        c->xalign = xalign;
        c->frame_rows = rows;
        ensure_partials(c);
    });
}

int fdtd_autotune(fdtd_ctx* c, int32_t steps_per_trial, int32_t* best_rows,
                  int32_t* best_zchunk) {
    if (!c) return FDTD_EINVAL;
    if (c->batch_owned) {
        c->err = "instance is stepped by its batch";
        return FDTD_ESTATE;
    }
    return guarded(c, [&] {
        need(steps_per_trial >= 1 && steps_per_trial <= 1000, "steps_per_trial out of range");
        need(c->kernel == FDTD_KERNEL_FUSED, "autotune applies to the fused kernel");
        ensure_time_tables(c, c->step + 2);
        // Trials read the live parity buffer and write the other one, which
        // the next real step overwrites: the state is left as it was.
        Problem q = c->p;
        q.diag_mask = 0;
        q.rec = nullptr;
        const int nz = c->p.nz;
        std::vector<int> chunks = {0};
        for (int d = 2; d <= 16; d *= 2)
            if (nz / d >= 8) chunks.push_back((nz + d - 1) / d);
        {
            int cus = 256;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
            for (int rows : {4, 8}) {
                const int dz = fused_default_zchunk(c->p, rows, c->xalign, cus);
                if (std::find(chunks.begin(), chunks.end(), dz) == chunks.end())
                    chunks.push_back(dz);
            }
        }
        // Whatever way the tuning ends, the profiler the trials detach comes
        // back and the events go; if it ends with an error part-way, the
        // settings and the energy mask the trials replaced are put back and
        // an intermediate buffer this call allocated is freed.
        struct Restore {
            fdtd_ctx* c;
            int rows, zchunk, frame, xalign, frame_rows, time_block, tb_rows, tb_zchunk;
            unsigned mask;
            EventTimer* timer;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            float *sf = nullptr, *sp = nullptr;   // scratch fields / CPML memories
            bool done = false;
            ~Restore() {
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                c->timer = timer;
                if (sf || sp) {
                    (void)hipStreamSynchronize(c->stream);
                    dfree(c, sf);
                    dfree(c, sp);
                }
                if (done) return;
                c->rows = rows;
                c->zchunk = zchunk;
                c->frame = frame;
                c->xalign = xalign;
                c->frame_rows = frame_rows;
                c->time_block = time_block;
                c->tb_rows = tb_rows;
                c->tb_zchunk = tb_zchunk;
                c->mask = mask;
                (void)hipStreamSynchronize(c->stream);
                try {
                    ensure_partials(c);
                } catch (...) {
                }
            }
        } rs{c, c->rows, c->zchunk, c->frame, c->xalign, c->frame_rows, c->time_block,
             c->tb_rows, c->tb_zchunk, c->mask, c->timer};
        check(hipEventCreate(&rs.e0), "event");
        check(hipEventCreate(&rs.e1), "event");
        const hipEvent_t e0 = rs.e0, e1 = rs.e1;
        // One-step trials step the way a run does, each reading what the
        // previous one wrote (re-running one step on unchanged inputs times
        // faster than stepping on small grids): the first trial launch writes
        // the free parity from the live state, and the later ones go back and
        // forth between the free parity and a scratch set of fields and CPML
        // memories, so the live state is never written. Without the memory
        // for the scratch set every launch re-runs the first.
        {
            const size_t nf = 6 * (size_t)c->p.fstride;
            const size_t np = c->p.npml > 0 ? psi_total(c->p) : 0;
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                free_b > (nf + np) * sizeof(float) + ((size_t)1 << 30)) {
                rs.sf = dalloc<float>(c, nf);
                rs.sp = dalloc<float>(c, np);
            }
        }
        Problem qa = q;   // index 0: the free parity, 1: the scratch set
        qa.fbase[0] = c->p.fbase[c->parity ^ 1];
        qa.fbase[1] = rs.sf;
        qa.pbase[0] = c->p.pbase[c->parity ^ 1];
        qa.pbase[1] = rs.sp;
        long long tcalls = 0;
        auto one_step_trial = [&] {
            if (!rs.sf || tcalls == 0)
                check(launch_step(c, q, c->step, c->parity, nullptr), "trial");
            else
                check(launch_step(c, qa, c->step, (int)((tcalls - 1) & 1), nullptr), "trial");
            ++tcalls;
        };
        // Milliseconds per step of `launch(steps)` (each call advancing
        // `per_call` steps): one untimed call, then at least steps_per_trial
        // steps, repeated with more steps until the timed span reaches 2 ms
        // so that small grids are not timed on a handful of launches.
        auto per_step = [&](auto&& launch, int per_call) {
            launch();
            int calls = std::max(1, steps_per_trial / per_call);
            for (int round = 0; round < 3; ++round) {
                check(hipEventRecord(e0, c->stream), "event");
                for (int s = 0; s < calls; ++s) launch();
                check(hipEventRecord(e1, c->stream), "event");
                check(hipEventSynchronize(e1), "event");
                float ms = 0.f;
                check(hipEventElapsedTime(&ms, e0, e1), "event");
                if (ms >= 2.0f || calls >= 1000 / per_call)
                    return ms / (float)(calls * per_call);
                calls = std::min(1000 / per_call,
                                 (int)(calls * (2.5f / std::max(ms, 0.01f))) + 1);
            }
            check(hipEventRecord(e0, c->stream), "event");
            for (int s = 0; s < calls; ++s) launch();
            check(hipEventRecord(e1, c->stream), "event");
            check(hipEventSynchronize(e1), "event");
            float ms = 0.f;
            check(hipEventElapsedTime(&ms, e0, e1), "event");
            return ms / (float)(calls * per_call);
        };
        float best = 1e30f;
        int br = c->rows, bz = c->zchunk, bf = c->frame, ba = c->xalign, bfr = c->frame_rows;
        c->timer = nullptr;
        const int frames[5][3] = {{FDTD_FRAME_SPLIT, 32, 2}, {FDTD_FRAME_FUSED, 32, 2},
                                  {FDTD_FRAME_FUSED, 64, 2}, {FDTD_FRAME_FUSED, 32, 4},
                                  {FDTD_FRAME_FUSED, 64, 4}};
        for (const auto& fa : frames) {
            for (int rows : {4, 8}) {
                for (int cz : chunks) {
                    c->frame = fa[0];
                    c->xalign = fa[1];
                    c->frame_rows = fa[2];
                    c->rows = rows;
                    c->zchunk = cz;
                    ensure_frame_tiles(c);
                    const float ms = per_step(one_step_trial, 1);
                    if (ms < best) {
                        best = ms;
                        br = rows;
                        bz = cz;
                        bf = fa[0];
                        ba = fa[1];
                        bfr = fa[2];
                    }
                }
            }
        }
        c->rows = br;
        c->zchunk = bz;
        c->frame = bf;
        c->xalign = ba;
        c->frame_rows = bfr;
        ensure_partials(c);
        // the two- and three-step kernels (per step: half a pair, a third of
        // a triple)
        const bool try2 = !c->p.periodic;
        int bt = 1, btr = c->tb_rows, btz = c->tb_zchunk;
        if (try2) {
            c->mask &= ~(unsigned)FDTD_DIAG_ENERGY;   // the trials run pairs and triples
            c->time_block = 2;
            // 8 or 16 chunks (each XCD then marches whole chunk layers of
            // tiles), 4, 2 (short grids: z slabs), and the whole z
            std::vector<int> chunks2;
            for (int cz : {(nz + 7) / 8, (nz + 15) / 16, (nz + 3) / 4, (nz + 1) / 2, 0})
                if (std::find(chunks2.begin(), chunks2.end(), cz) == chunks2.end())
                    chunks2.push_back(cz);
            for (int steps : {2, 3}) {
                c->time_block = steps;
                for (int rows : {4, 2}) {
                    for (int cz : chunks2) {
                        if (cz > nz) continue;
                        c->tb_rows = rows;
                        c->tb_zchunk = cz;
                        const float ms =
                            steps == 3
                                ? per_step([&] { launch_triple(c, c->step, true); }, 3)
                                : per_step([&] { launch_pair(c, c->step, true); }, 2);
                        if (ms < best) {
                            best = ms;
                            bt = steps;
                            btr = rows;
                            btz = cz;
                        }
                    }
                }
            }
            c->mask = rs.mask;
            c->time_block = rs.time_block;
            c->tb_rows = rs.tb_rows;
            c->tb_zchunk = rs.tb_zchunk;
        }
        if (bt >= 2) {
            c->time_block = bt;
            c->tb_rows = btr;
            c->tb_zchunk = btz;
        } else {
            c->time_block = 1;
        }
        rs.done = true;
        if (best_rows) *best_rows = br;
        if (best_zchunk) *best_zchunk = bz;
    });
}

int fdtd_profile_enable(fdtd_ctx* c, int32_t on) {
    if (!c) return FDTD_EINVAL;
    return guarded(c, [&] {
        check(hipStreamSynchronize(c->stream), "sync");
        delete c->timer;
        c->timer = nullptr;
        if (on) {
            c->timer = new EventTimer();
            c->timer->stream = c->stream;
        }
    });
}

int fdtd_profile_read(fdtd_ctx* c, fdtd_kernel_profile* out, int32_t max, int32_t* count) {
    if (!c || !count || max < 0 || (max > 0 && !out)) return FDTD_EINVAL;
    return guarded(c, [&] {
        need(c->timer != nullptr, "profiling is off", FDTD_ESTATE);
        check(hipStreamSynchronize(c->stream), "sync");
        c->timer->collect();
        const auto& t = c->timer->totals;
        *count = (int32_t)t.size();
        for (int32_t i = 0; i < max && i < (int32_t)t.size(); ++i) {
            std::memset(out[i].name, 0, sizeof out[i].name);
            std::strncpy(out[i].name, t[i].first.c_str(), sizeof out[i].name - 1);
            out[i].launches = t[i].second.first;
            out[i].total_ms = t[i].second.second;
        }
    });
}

}  // extern "C"
