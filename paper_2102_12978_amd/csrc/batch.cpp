// Batch of independent solver instances advanced together: one E launch and
// one H launch per step over a flattened work list (kernels_batch.hip), with
// runs of steps replayed from captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "context.hpp"

using namespace bfdtd;

struct fdtd_batch {
    hipStream_t stream = nullptr;      // caller's stream: uploads, graph and eager launches
    hipStream_t capture = nullptr;     // private stream used only to record graphs
    std::vector<fdtd_ctx*> inst;
    std::vector<Problem> host_probs;
    Problem* probs = nullptr;          // device copy of every instance's Problem
    long long* nctr = nullptr;         // device step counter read by the kernels
    int4* work = nullptr;
    int nwork = 0;
    int cols = 256, zchunk = 1, blocks = 0;
    int planes = 0;                    // split kernels with zchunk 1: one block per plane
    int kernel = FDTD_KERNEL_SPLIT;    // split E/H passes, or fused boundary tiles
    int bnd_rows = 2;                  // rows per fused boundary tile (2 or 4)
    int graph_steps = 20;              // even, so a replay leaves the parity unchanged
    // two-step kernel (time_block 2): pairs of steps, four tile-class launches
    int time_block = 1, tb_rows = 2, tb_zchunk = 16;
    int4* items2 = nullptr;            // the four classes' work items, back to back
    int nitems2[4] = {0, 0, 0, 0};
    SideStreams side{};                // the boundary classes' launches beside the interior
    bool side_ok = false;
    long long items2_bytes = 0;
    hipGraphExec_t exec[2] = {nullptr, nullptr};   // per starting parity
    int cu_count = 256;
    long long step = 0;
    int parity = 0;
    long long device_bytes = 0;
    std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

void drop_graphs(fdtd_batch* b) {
    for (auto& e : b->exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
}

template <typename F>
int bguard(fdtd_batch* b, F&& f) {
    try {
        f();
        return FDTD_OK;
    } catch (const Fail& e) {
        if (b) b->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (b) b->err = "host allocation failed";
        return FDTD_ENOMEM;
    } catch (...) {
        if (b) b->err = "unexpected exception";
        return FDTD_EDEVICE;
    }
}

void* balloc(fdtd_batch* b, size_t bytes) {
    void* p = nullptr;
    check(hipMalloc(&p, bytes), "hipMalloc");
    b->device_bytes += (long long)bytes;
    return p;
}

// z chunk of the fused tiles (0: whole z, i.e. larger than any instance)
int fused_cz(const fdtd_batch* b) { return b->zchunk > 0 ? b->zchunk : (1 << 30); }

// Work items. Split kernels: per instance, blocks of `cols` flattened (x, y)
// columns (x running over the padded pitch) times z ranges of `zchunk`
// planes (0: the whole z extent). Fused kernel: per instance and z chunk,
// tiles of 64 x cells by bnd_rows rows, x fastest so that consecutive tiles
// are x-adjacent.
void build_work(fdtd_batch* b) {
    std::vector<int4> w;
    for (int q = 0; q < (int)b->inst.size(); ++q) {
        const Problem& p = b->inst[q]->p;
        if (b->kernel == FDTD_KERNEL_FUSED) {
            const int cz = std::min(fused_cz(b), p.nz);
            for (int c = 0; c * cz < p.nz; ++c)
                for (int y0 = 0; y0 < p.ny; y0 += b->bnd_rows)
                    for (int x0 = 0; x0 < p.nx; x0 += 64) w.push_back(make_int4(q, x0, y0, c));
            continue;
        }
        const int ncol = p.pitch * p.ny;   // columns over the padded pitch (x >= nx idle)
        if (b->zchunk == 1) {              // plane grid: the kernels take k from the grid
            for (int c0 = 0; c0 < ncol; c0 += b->cols) w.push_back(make_int4(q, c0, 0, 1));
            continue;
        }
        const int zc = b->zchunk > 0 ? std::min(b->zchunk, p.nz) : p.nz;
        for (int c0 = 0; c0 < ncol; c0 += b->cols)
            for (int k0 = 0; k0 < p.nz; k0 += zc) w.push_back(make_int4(q, c0, k0, std::min(k0 + zc, p.nz)));
    }
    b->planes = 0;
    if (b->kernel != FDTD_KERNEL_FUSED && b->zchunk == 1)
        for (const auto& c : b->inst) b->planes = std::max(b->planes, c->p.nz);
    need(b->planes <= 65535, "z extent too large for a per-plane grid");
    need(w.size() < (size_t)1 << 30, "too many work items");
    check(hipStreamSynchronize(b->stream), "sync");
    drop_graphs(b);
    if (b->work) {
        (void)hipFree(b->work);
        b->device_bytes -= (long long)b->nwork * (long long)sizeof(int4);
        b->work = nullptr;
    }
    b->nwork = (int)w.size();
    b->work = static_cast<int4*>(balloc(b, w.size() * sizeof(int4)));
    check(hipMemcpy(b->work, w.data(), w.size() * sizeof(int4), hipMemcpyHostToDevice), "copy work");
    // persistent grid: as many workgroups as can be resident at once
    if (b->kernel == FDTD_KERNEL_FUSED) {
        const int per_cu = fused_bnd_blocks_per_cu(b->bnd_rows, true);
        b->blocks = std::max(1, std::min((b->nwork + 3) / 4, b->cu_count * per_cu));
    } else {
        const int per_cu = batch_blocks_per_cu(b->cols);
        b->blocks = std::max(1, std::min(b->nwork, b->cu_count * per_cu));
    }
}

// Push every instance's Problem (with its diagnostics selection) to the
// device when it differs from the copy already there. The copy waits for
// the stream first: launches still queued read the old copy.
void upload_problems(fdtd_batch* b, bool force = false) {
    std::vector<Problem> now(b->inst.size());
    for (size_t q = 0; q < b->inst.size(); ++q) {
        const fdtd_ctx* c = b->inst[q];
        std::memcpy(&now[q], &c->p, sizeof(Problem));
        now[q].plane = c->plane;
        now[q].diag_mask = c->plane >= 0 ? (int)(c->mask & 7u) : 0;
        now[q].win_begin = c->wbegin;
        now[q].rec = nullptr;
    }
    if (!force && std::memcmp(now.data(), b->host_probs.data(), now.size() * sizeof(Problem)) == 0)
        return;
    check(hipStreamSynchronize(b->stream), "sync");
    b->host_probs = now;
    check(hipMemcpy(b->probs, b->host_probs.data(), b->host_probs.size() * sizeof(Problem),
                    hipMemcpyHostToDevice), "copy problems");
}

// Work items of the two-step kernel for the current instances and tile.
void build_items2(fdtd_batch* b) {
    std::vector<Problem> ps;
    for (const fdtd_ctx* c : b->inst) ps.push_back(c->p);
    for (const Problem& p : ps) need(p.nz < 65536, "z extent too large for the two-step items");
    std::vector<int4> it[4];
    step2_batch_items(ps, b->tb_rows, b->tb_zchunk, it);
    std::vector<int4> all;
    for (int c = 0; c < 4; ++c) {
        b->nitems2[c] = (int)it[c].size();
        all.insert(all.end(), it[c].begin(), it[c].end());
    }
    check(hipStreamSynchronize(b->stream), "sync");
    drop_graphs(b);
    if (b->items2) {
        (void)hipFree(b->items2);
        b->device_bytes -= b->items2_bytes;
        b->items2 = nullptr;
        b->items2_bytes = 0;
    }
    b->items2_bytes = (long long)(std::max<size_t>(1, all.size()) * sizeof(int4));
    b->items2 = static_cast<int4*>(balloc(b, (size_t)b->items2_bytes));
    if (!all.empty())
        check(hipMemcpy(b->items2, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice),
              "copy items");
}

// One pair of steps of every instance through the two-step kernel.
hipError_t launch_two(const fdtd_batch* b, hipStream_t s, int off, int par, int diag) {
    const int4* it[4];
    long long o = 0;
    for (int c = 0; c < 4; ++c) {
        it[c] = b->items2 + o;
        o += b->nitems2[c];
    }
    return launch_step2_batch(b->probs, it, b->nitems2, b->tb_rows, b->nctr, off, par, diag, s,
                              b->side_ok ? &b->side : nullptr);
}

hipError_t launch_pair(const fdtd_batch* b, hipStream_t s, int off, int par, int diag) {
    if (b->kernel == FDTD_KERNEL_FUSED)
        return launch_fused_bnd(b->host_probs[0], b->probs, b->work, b->nwork, b->bnd_rows,
                                fused_cz(b), b->blocks, b->nctr, off, par, diag,
                                Frame{0, 0, 0, 0}, nullptr, s);
    hipError_t e = launch_batch_e(b->probs, b->work, b->nwork, b->cols, b->blocks, b->planes,
                                  b->nctr, off, par, diag, s);
    if (e != hipSuccess) return e;
    return launch_batch_h(b->probs, b->work, b->nwork, b->cols, b->blocks, b->planes, b->nctr,
                          off, par, s);
}

// Record graph_steps steps starting at parity par, then the counter advance.
void capture_graph(fdtd_batch* b, int par) {
    hipGraph_t g = nullptr;
    check(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed), "begin capture");
    hipError_t le = hipSuccess;
    if (b->time_block == 2) {
        for (int i = 0; 2 * i < b->graph_steps && le == hipSuccess; ++i)
            le = launch_two(b, b->capture, 2 * i, (par + i) & 1, 1);
    } else {
        for (int i = 0; i < b->graph_steps && le == hipSuccess; ++i)
            le = launch_pair(b, b->capture, i, (par + i) & 1, 1);
    }
    if (le == hipSuccess) le = launch_batch_advance(b->nctr, b->graph_steps, b->capture);
    hipError_t ee = hipStreamEndCapture(b->capture, &g);
    check(le, "captured launch");
    check(ee, "end capture");
    hipError_t ie = hipGraphInstantiate(&b->exec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check(ie, "graph instantiate");
}

void after_steps(fdtd_batch* b, long long n0, long long nsteps) {
    for (fdtd_ctx* c : b->inst) {
        if (c->plane >= 0 && (c->mask & 7u)) {
            const long long first = std::max(n0, c->wbegin);
            if (n0 + nsteps > first) c->count += n0 + nsteps - first;
        }
        c->step = n0 + nsteps;
        c->parity = b->parity;
        c->energy_valid = false;
    }
}

}  // namespace

extern "C" {

int fdtd_batch_create(int32_t count, const fdtd_grid* grids, const fdtd_injector* injectors,
                      void* stream, fdtd_batch** out) {
    if (!out) return FDTD_EINVAL;
    *out = nullptr;
    if (count < 1 || !grids) {
        g_batch_create_error = "need count >= 1 and a grid array";
        return FDTD_EINVAL;
    }
    fdtd_batch* b = new (std::nothrow) fdtd_batch();
    if (!b) {
        g_batch_create_error = "host allocation failed";
        return FDTD_ENOMEM;
    }
    b->stream = (hipStream_t)stream;
    int rc = bguard(b, [&] {
        int dev = 0;
        check(hipGetDevice(&dev), "hipGetDevice");
        check(hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev),
              "CU count");
        check(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
        create_side_streams(b->side);
        b->side_ok = true;
        for (int q = 0; q < count; ++q) {
            fdtd_grid g = grids[q];
            g.stream = stream;
            g.kernel = FDTD_KERNEL_SPLIT;
            fdtd_ctx* c = nullptr;
            int r = fdtd_create(&g, &c);
            if (r != FDTD_OK)
                throw Fail{r, "instance " + std::to_string(q) + ": " + fdtd_last_error(nullptr)};
            c->batch_owned = true;
            b->inst.push_back(c);
            if (injectors) {
                r = fdtd_set_injector(c, &injectors[q]);
                if (r != FDTD_OK)
                    throw Fail{r, "instance " + std::to_string(q) + ": " + c->err};
            }
        }
        b->host_probs.resize(count);
        b->probs = static_cast<Problem*>(balloc(b, count * sizeof(Problem)));
        b->nctr = static_cast<long long*>(balloc(b, sizeof(long long)));
        check(hipMemsetAsync(b->nctr, 0, sizeof(long long), b->stream), "clear counter");
        build_work(b);
        upload_problems(b, true);
        check(hipStreamSynchronize(b->stream), "sync");
    });
    if (rc != FDTD_OK) {
        g_batch_create_error = b->err;
        fdtd_batch_destroy(b);
        return rc;
    }
    *out = b;
    return FDTD_OK;
}

int fdtd_batch_destroy(fdtd_batch* b) {
    if (!b) return FDTD_OK;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (fdtd_ctx* c : b->inst) {
        c->batch_owned = false;
        fdtd_destroy(c);
    }
    if (b->probs) (void)hipFree(b->probs);
    if (b->nctr) (void)hipFree(b->nctr);
    if (b->work) (void)hipFree(b->work);
    if (b->items2) (void)hipFree(b->items2);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    release_side_streams(b->side);
    delete b;
    return FDTD_OK;
}

const char* fdtd_batch_last_error(const fdtd_batch* b) {
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

fdtd_ctx* fdtd_batch_instance(fdtd_batch* b, int32_t q) {
    if (!b || q < 0 || q >= (int)b->inst.size()) return nullptr;
    return b->inst[q];
}

int fdtd_batch_step(fdtd_batch* b, int64_t nsteps) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(nsteps >= 0, "nsteps must be >= 0");
        if (nsteps == 0) return;
        for (fdtd_ctx* c : b->inst) ensure_time_tables(c, b->step + nsteps + 1);
        upload_problems(b);
        const long long n0 = b->step;
        long long left = nsteps;
        if (b->graph_steps > 0) {
            while (left >= b->graph_steps) {
                if (!b->exec[b->parity]) capture_graph(b, b->parity);
                check(hipGraphLaunch(b->exec[b->parity], b->stream), "graph launch");
                left -= b->graph_steps;
            }
        }
        for (; left > 0;) {
            if (b->time_block == 2 && left >= 2) {
                check(launch_two(b, b->stream, 0, b->parity, 1), "batch launch");
                check(launch_batch_advance(b->nctr, 2, b->stream), "counter advance");
                left -= 2;
            } else {
                check(launch_pair(b, b->stream, 0, b->parity, 1), "batch launch");
                check(launch_batch_advance(b->nctr, 1, b->stream), "counter advance");
                left -= 1;
            }
            b->parity ^= 1;
        }
        b->step = n0 + nsteps;
        after_steps(b, n0, nsteps);
    });
}

int fdtd_batch_set_tile(fdtd_batch* b, int32_t cols, int32_t zchunk) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(cols == 64 || cols == 128 || cols == 256, "cols must be 64, 128 or 256");
        need(zchunk >= 0, "zchunk must be >= 0");
        b->cols = cols;
        b->zchunk = zchunk;
        build_work(b);
    });
}

int fdtd_batch_set_kernel(fdtd_batch* b, int32_t kernel, int32_t rows) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(kernel == FDTD_KERNEL_FUSED || kernel == FDTD_KERNEL_SPLIT,
             "kernel must be FDTD_KERNEL_FUSED or FDTD_KERNEL_SPLIT");
        need(rows == 2 || rows == 4, "rows must be 2 or 4");
        b->kernel = kernel;
        b->bnd_rows = rows;
        build_work(b);
    });
}

int fdtd_batch_set_time_block(fdtd_batch* b, int32_t steps, int32_t rows, int32_t zchunk) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(steps == 1 || steps == 2, "steps must be 1 or 2");
        need(rows == 2 || rows == 4, "rows must be 2 or 4");
        need(zchunk >= 0, "zchunk must be >= 0");
        for (const fdtd_ctx* c : b->inst)
            need(!c->p.periodic, "the two-step kernel does not run the periodic test mode");
        b->tb_rows = rows;
        b->tb_zchunk = zchunk;
        if (steps == 2) build_items2(b);
        check(hipStreamSynchronize(b->stream), "sync");
        drop_graphs(b);
        b->time_block = steps;
    });
}

int fdtd_batch_set_graph_steps(fdtd_batch* b, int32_t steps) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(steps == 0 || (steps >= 2 && steps % 2 == 0 && steps <= 1000),
             "graph steps must be 0 or an even number in [2, 1000]");
        check(hipStreamSynchronize(b->stream), "sync");
        drop_graphs(b);
        b->graph_steps = steps;
    });
}

int fdtd_batch_autotune(fdtd_batch* b, int32_t steps_per_trial, int32_t* best_cols,
                        int32_t* best_zchunk) {
    if (!b) return FDTD_EINVAL;
    return bguard(b, [&] {
        need(steps_per_trial >= 1 && steps_per_trial <= 1000, "steps_per_trial out of range");
        for (fdtd_ctx* c : b->inst) ensure_time_tables(c, b->step + 1);
        upload_problems(b);
        hipEvent_t e0, e1;
        check(hipEventCreate(&e0), "event");
        check(hipEventCreate(&e1), "event");
        int bk = b->kernel, bc = b->cols, bz = b->zchunk, br = b->bnd_rows;
        float best = -1.f;
        struct Cand { int kernel, cols, zc, rows; };
        std::vector<Cand> cands;
        for (int rows : {2, 4})
            for (int zc : {0, 32, 16, 8}) cands.push_back({FDTD_KERNEL_FUSED, b->cols, zc, rows});
        for (int cols : {64, 128, 256})
            for (int zc : {0, 16, 8, 4, 1}) cands.push_back({FDTD_KERNEL_SPLIT, cols, zc, br});
        // Trials read the live parity and write the other one only, with the
        // plane accumulation off, so the state is left as it was.
        for (const Cand& cd : cands) {
            b->kernel = cd.kernel;
            b->bnd_rows = cd.rows;
            b->cols = cd.cols;
            b->zchunk = cd.zc;
            build_work(b);
            check(launch_pair(b, b->stream, 0, b->parity, 0), "trial");
            check(hipEventRecord(e0, b->stream), "event");
            for (int t = 0; t < steps_per_trial; ++t)
                check(launch_pair(b, b->stream, 0, b->parity, 0), "trial");
            check(hipEventRecord(e1, b->stream), "event");
            check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (best < 0.f || ms < best) {
                best = ms;
                bk = cd.kernel;
                bc = cd.cols;
                bz = cd.zc;
                br = cd.rows;
            }
        }
        // the two-step kernel (per step: half a pair), except for periodic
        // instances
        bool periodic = false;
        for (const fdtd_ctx* c : b->inst) periodic = periodic || c->p.periodic;
        int bt = 1, btr = b->tb_rows, btz = b->tb_zchunk;
        if (!periodic) {
            const int rows0 = b->tb_rows, zc0 = b->tb_zchunk;
            for (int rows : {2, 4})
                for (int zc : {16, 32, 8, 0}) {
                    b->tb_rows = rows;
                    b->tb_zchunk = zc;
                    build_items2(b);
                    check(launch_two(b, b->stream, 0, b->parity, 0), "trial");
                    const int pairs = std::max(1, steps_per_trial / 2);
                    check(hipEventRecord(e0, b->stream), "event");
                    for (int t = 0; t < pairs; ++t)
                        check(launch_two(b, b->stream, 0, b->parity, 0), "trial");
                    check(hipEventRecord(e1, b->stream), "event");
                    check(hipEventSynchronize(e1), "event sync");
                    float ms = 0.f;
                    check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
                    ms *= (float)steps_per_trial / (float)(2 * pairs);
                    if (ms < best) {
                        best = ms;
                        bt = 2;
                        btr = rows;
                        btz = zc;
                    }
                }
            b->tb_rows = rows0;
            b->tb_zchunk = zc0;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->kernel = bk;
        b->bnd_rows = br;
        b->cols = bc;
        b->zchunk = bz;
        build_work(b);
        b->tb_rows = btr;
        b->tb_zchunk = btz;
        if (bt == 2) build_items2(b);
        b->time_block = bt;
        if (best_cols) *best_cols = bk == FDTD_KERNEL_FUSED ? 0 : bc;
        if (best_zchunk) *best_zchunk = bz;
    });
}

int fdtd_batch_get_info(const fdtd_batch* b, fdtd_batch_info* out) {
    if (!b || !out) return FDTD_EINVAL;
    fdtd_batch_info r{};
    r.count = (int32_t)b->inst.size();
    long long bytes = b->device_bytes;
    for (const fdtd_ctx* c : b->inst) {
        r.cells += (int64_t)c->p.nx * c->p.ny * c->p.nz;
        bytes += c->device_bytes;
    }
    r.tile_cols = b->cols;
    r.tile_zchunk = b->zchunk;
    r.work_items = b->nwork;
    r.blocks = b->blocks;
    r.graph_steps = b->graph_steps;
    r.step = b->step;
    r.device_bytes = bytes;
    r.kernel = b->kernel;
    r.time_block = b->time_block;
    r.tb_rows = b->tb_rows;
    r.tb_zchunk = b->tb_zchunk;
    r.tb_items = b->nitems2[0] + b->nitems2[1] + b->nitems2[2] + b->nitems2[3];
    *out = r;
    return FDTD_OK;
}

}  // extern "C"
