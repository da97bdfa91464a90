// Two-kernel Yee step (one thread per cell): E update + E source, then
// H update + H source, each reading the old ping-pong buffer and writing the
// new one. It carries every boundary case (PEC walls, CPML slabs, periodic
// wrap) and moves 72 B per cell-update.
//
// The cells are enumerated as a flat list of (x, y) columns of a frame
// around an excluded rectangle (bottom rows y < y0, top rows y >= y1, then
// the left x < x0 and right x >= x1 strips of the rows in between); an empty
// rectangle makes the frame the whole grid.
#include <hip/hip_runtime.h>

#include "yee_cell.hpp"

namespace bfdtd {

namespace {

constexpr int BT = 256;

__device__ __forceinline__ void block_energy(double v, double* out) {
    __shared__ double red[BT / 64];
    v = wave_sum(v);
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// nd: cells inside this rectangle are updated without the plane
// accumulation (cells that another kernel owns and accumulates).
__global__ void __launch_bounds__(BT)
split_e_kernel(Problem p, long long n, int par, Frame fr, long long ncols, double* epart,
               Frame nd) {
    int i = 0, j = 0;
    const int k = blockIdx.y;
    const unsigned col = blockIdx.x * BT + threadIdx.x;
    const bool inside = col < (unsigned long long)ncols && frame_column(fr, p.nx, p.ny, col, &i, &j);
    const bool owned = !(i >= nd.x0 && i < nd.x1 && j >= nd.y0 && j < nd.y1);
    const double e2 = inside ? e_point(p, n, par, i, j, k, owned ? p.diag_mask : 0) : 0.0;
    if (epart) block_energy(e2, epart + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ void __launch_bounds__(BT)
split_h_kernel(Problem p, long long n, int par, Frame fr, long long ncols, double* epart) {
    int i = 0, j = 0;
    const int k = blockIdx.y;
    const unsigned col = blockIdx.x * BT + threadIdx.x;
    const bool inside = col < (unsigned long long)ncols && frame_column(fr, p.nx, p.ny, col, &i, &j);
    const double hh = inside ? h_point(p, n, par, i, j, k) : 0.0;
    if (epart) block_energy(hh, epart + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

}  // namespace

long long frame_columns(const Problem& p, const Frame& fr) {
    return (long long)fr.y0 * p.nx + (long long)(p.ny - fr.y1) * p.nx +
           (long long)(fr.y1 - fr.y0) * (fr.x0 + p.nx - fr.x1);
}

int split_partial_count(const Problem& p, const Frame& fr) {
    const long long nc = frame_columns(p, fr);
    return nc == 0 ? 0 : 2 * (int)((nc + BT - 1) / BT) * p.nz;
}

hipError_t launch_split_frame(const Problem& p, long long n, int parity, const Frame& fr,
                              double* epart, hipStream_t s, LaunchTimer* timer) {
    const long long nc = frame_columns(p, fr);
    if (nc == 0) return hipSuccess;
    dim3 grid((unsigned)((nc + BT - 1) / BT), p.nz, 1);
    const size_t nb = (size_t)grid.x * grid.y;
    if (timer) timer->mark(fr.x1 > 0 ? "frame_e" : "split_e");
    hipLaunchKernelGGL(split_e_kernel, grid, dim3(BT), 0, s, p, n, parity, fr, nc, epart,
                       Frame{0, 0, 0, 0});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timer) timer->mark(fr.x1 > 0 ? "frame_h" : "split_h");
    hipLaunchKernelGGL(split_h_kernel, grid, dim3(BT), 0, s, p, n, parity, fr, nc,
                       epart ? epart + nb : nullptr);
    if (timer) timer->mark(nullptr);
    return hipGetLastError();
}

}  // namespace bfdtd
