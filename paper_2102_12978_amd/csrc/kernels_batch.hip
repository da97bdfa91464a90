// Batched Yee step over many independent instances of uneven size. All
// instances advance in lockstep: one E launch and one H launch per step walk
// a single flattened list of work items (instance, block of flattened (x, y)
// columns over the padded row pitch, so that a wavefront reads one aligned
// 256-byte row segment, z range) with a persistent grid, so small instances
// do not leave the chip idle and the whole step is two launches regardless of the
// instance count. The per-cell arithmetic is the split kernels' (every
// boundary case, the antenna source and the plane accumulation), so an
// instance advances bit-identically to a single-domain split-kernel run.
//
// The step index comes from a device counter (plus a per-launch offset) so
// that a captured multi-step graph stays valid when replayed; a one-thread
// kernel advances the counter at the end of each replay.
#include <hip/hip_runtime.h>

#include "yee_cell.hpp"

namespace bfdtd {

namespace {

constexpr int MAX_COLS = 256;

// The parity is a template argument so that the copied Problem is indexed
// with constants only and stays in registers.
template <int par>
__global__ void __launch_bounds__(MAX_COLS)
batch_e_kernel(const Problem* __restrict__ probs, const int4* __restrict__ work, int nwork,
               const long long* __restrict__ nctr, int off, int diag) {
    const long long n = *nctr + off;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int4 wk = work[w];
        const Problem p = probs[wk.x];   // a copy: stores below cannot alias it
        const int col = wk.y + (int)threadIdx.x;
        const int i = col % p.pitch, j = col / p.pitch;
        if (i >= p.nx || j >= p.ny) continue;
        const int mask = (diag && n >= p.win_begin) ? p.diag_mask : 0;
        for (int k = wk.z; k < wk.w; ++k) (void)e_point(p, n, par, i, j, k, mask);
    }
}

template <int par>
__global__ void __launch_bounds__(MAX_COLS)
batch_h_kernel(const Problem* __restrict__ probs, const int4* __restrict__ work, int nwork,
               const long long* __restrict__ nctr, int off) {
    const long long n = *nctr + off;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int4 wk = work[w];
        const Problem p = probs[wk.x];
        const int col = wk.y + (int)threadIdx.x;
        const int i = col % p.pitch, j = col / p.pitch;
        if (i >= p.nx || j >= p.ny) continue;
        for (int k = wk.z; k < wk.w; ++k) (void)h_point(p, n, par, i, j, k);
    }
}

// One workgroup per (column block, plane): block x is the work item (its
// k range unused), block y the plane; planes past an instance's nz exit.
// No loop, so every cell's loads are in flight at once across the grid.
template <int par>
__global__ void __launch_bounds__(MAX_COLS)
batch_e_plane_kernel(const Problem* __restrict__ probs, const int4* __restrict__ work,
                     const long long* __restrict__ nctr, int off, int diag) {
    const long long n = *nctr + off;
    const int4 wk = work[blockIdx.x];
    const Problem p = probs[wk.x];
    const int k = blockIdx.y;
    const int col = wk.y + (int)threadIdx.x;
    const int i = col % p.pitch, j = col / p.pitch;
    if (k >= p.nz || i >= p.nx || j >= p.ny) return;
    const int mask = (diag && n >= p.win_begin) ? p.diag_mask : 0;
    (void)e_point(p, n, par, i, j, k, mask);
}

template <int par>
__global__ void __launch_bounds__(MAX_COLS)
batch_h_plane_kernel(const Problem* __restrict__ probs, const int4* __restrict__ work,
                     const long long* __restrict__ nctr, int off) {
    const long long n = *nctr + off;
    const int4 wk = work[blockIdx.x];
    const Problem p = probs[wk.x];
    const int k = blockIdx.y;
    const int col = wk.y + (int)threadIdx.x;
    const int i = col % p.pitch, j = col / p.pitch;
    if (k >= p.nz || i >= p.nx || j >= p.ny) return;
    (void)h_point(p, n, par, i, j, k);
}

__global__ void batch_advance_kernel(long long* nctr, int by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) nctr[0] += by;
}

}  // namespace

hipError_t launch_batch_e(const Problem* probs, const int4* work, int nwork, int cols, int blocks,
                          int planes, const long long* nctr, int off, int par, int diag,
                          hipStream_t s) {
    if (cols < 1 || cols > MAX_COLS || blocks < 1) return hipErrorInvalidValue;
    if (planes > 0) {
        const dim3 g((unsigned)nwork, (unsigned)planes);
        if (par)
            hipLaunchKernelGGL(batch_e_plane_kernel<1>, g, dim3(cols), 0, s, probs, work, nctr,
                               off, diag);
        else
            hipLaunchKernelGGL(batch_e_plane_kernel<0>, g, dim3(cols), 0, s, probs, work, nctr,
                               off, diag);
        return hipGetLastError();
    }
    if (par)
        hipLaunchKernelGGL(batch_e_kernel<1>, dim3(blocks), dim3(cols), 0, s, probs, work, nwork,
                           nctr, off, diag);
    else
        hipLaunchKernelGGL(batch_e_kernel<0>, dim3(blocks), dim3(cols), 0, s, probs, work, nwork,
                           nctr, off, diag);
    return hipGetLastError();
}

hipError_t launch_batch_h(const Problem* probs, const int4* work, int nwork, int cols, int blocks,
                          int planes, const long long* nctr, int off, int par, hipStream_t s) {
    if (cols < 1 || cols > MAX_COLS || blocks < 1) return hipErrorInvalidValue;
    if (planes > 0) {
        const dim3 g((unsigned)nwork, (unsigned)planes);
        if (par)
            hipLaunchKernelGGL(batch_h_plane_kernel<1>, g, dim3(cols), 0, s, probs, work, nctr,
                               off);
        else
            hipLaunchKernelGGL(batch_h_plane_kernel<0>, g, dim3(cols), 0, s, probs, work, nctr,
                               off);
        return hipGetLastError();
    }
    if (par)
        hipLaunchKernelGGL(batch_h_kernel<1>, dim3(blocks), dim3(cols), 0, s, probs, work, nwork,
                           nctr, off);
    else
        hipLaunchKernelGGL(batch_h_kernel<0>, dim3(blocks), dim3(cols), 0, s, probs, work, nwork,
                           nctr, off);
    return hipGetLastError();
}

int batch_blocks_per_cu(int cols) {
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, batch_e_kernel<0>, cols, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_h_kernel<0>, cols, 0) != hipSuccess)
        return 1;
    return a < b ? (a > 0 ? a : 1) : (b > 0 ? b : 1);
}

hipError_t launch_batch_advance(long long* nctr, int by, hipStream_t s) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, s, nctr, by);
    return hipGetLastError();
}

}  // namespace bfdtd
