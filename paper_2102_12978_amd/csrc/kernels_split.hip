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

__device__ __forceinline__ bool frame_column(const Frame& fr, int nx, int ny, long long c, int* x,
                                             int* y) {
    const long long nb = (long long)fr.y0 * nx;
    const long long nt = (long long)(ny - fr.y1) * nx;
    const long long nl = (long long)(fr.y1 - fr.y0) * fr.x0;
    const long long nr = (long long)(fr.y1 - fr.y0) * (nx - fr.x1);
    if (c < nb) {
        *y = (int)(c / nx);
        *x = (int)(c % nx);
    } else if ((c -= nb) < nt) {
        *y = fr.y1 + (int)(c / nx);
        *x = (int)(c % nx);
    } else if ((c -= nt) < nl) {
        *y = fr.y0 + (int)(c / fr.x0);
        *x = (int)(c % fr.x0);
    } else if ((c -= nl) < nr) {
        const int wdt = nx - fr.x1;
        *y = fr.y0 + (int)(c / wdt);
        *x = fr.x1 + (int)(c % wdt);
    } else {
        return false;
    }
    return true;
}

__global__ void __launch_bounds__(BT)
split_e_kernel(Problem p, long long n, int par, Frame fr, long long ncols, double* epart) {
    int i = 0, j = 0;
    const int k = blockIdx.y;
    const long long col = (long long)blockIdx.x * BT + threadIdx.x;
    const bool inside = col < ncols && frame_column(fr, p.nx, p.ny, col, &i, &j);
    double e2 = 0.0;
    if (inside) {
        auto fo = [&](int c) -> const float* { return fptr(p, par, c); };
        auto fn = [&](int c) -> float* { return fptr(p, par ^ 1, c); };
        const bool per = p.periodic != 0;
        const int km = k == 0 ? p.nz - 1 : k - 1;
        int im = i - 1, jm = j - 1;
        const bool has_im = im >= 0 || per, has_jm = jm >= 0 || per;
        if (im < 0) im += p.nx;
        if (jm < 0) jm += p.ny;
        const size_t row = ((size_t)k * p.ny + j) * p.pitch;
        const size_t row_jm = ((size_t)k * p.ny + jm) * p.pitch;
        const size_t row_km = ((size_t)km * p.ny + j) * p.pitch;
        const size_t id = row + i;
        HNbr h;
        h.hx = fo(HX)[id];
        h.hy = fo(HY)[id];
        h.hz = fo(HZ)[id];
        h.hz_im = has_im ? fo(HZ)[row + im] : 0.f;
        h.hy_im = has_im ? fo(HY)[row + im] : 0.f;
        h.hz_jm = has_jm ? fo(HZ)[row_jm + i] : 0.f;
        h.hx_jm = has_jm ? fo(HX)[row_jm + i] : 0.f;
        h.hy_km = fo(HY)[row_km + i];
        h.hx_km = fo(HX)[row_km + i];
        float ex = fo(EX)[id], ey = fo(EY)[id], ez = fo(EZ)[id];
        const int slot = p.colmap ? p.colmap[(size_t)j * p.nx + i] : -1;
        float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
        if (slot >= 0) {
            const float2 t = p.tE[n];
            pt0 = cmul(p.zph[2 * k], t);
            pt1 = cmul(p.zph[2 * k + 1], t);
        }
        e_cell(p, par, i, j, k, h, ex, ey, ez, slot, pt0, pt1, true);
        fn(EX)[id] = ex;
        fn(EY)[id] = ey;
        fn(EZ)[id] = ez;
        if (k == p.plane) {
            const size_t pl = (size_t)j * p.nx + i, ps = (size_t)p.nx * p.ny;
            if (p.diag_mask & FDTD_DIAG_EX2) p.fl[pl] += (double)ex * ex;
            if (p.diag_mask & FDTD_DIAG_EY2) p.fl[ps + pl] += (double)ey * ey;
            if (p.diag_mask & FDTD_DIAG_EZ2) p.fl[2 * ps + pl] += (double)ez * ez;
            if (p.rec) p.rec[(size_t)(n - p.rec_begin) * ps + pl] = ey;
        }
        e2 = (double)ex * ex + (double)ey * ey + (double)ez * ez;
    }
    if (epart) block_energy(e2, epart + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ void __launch_bounds__(BT)
split_h_kernel(Problem p, long long n, int par, Frame fr, long long ncols, double* epart) {
    int i = 0, j = 0;
    const int k = blockIdx.y;
    const long long col = (long long)blockIdx.x * BT + threadIdx.x;
    const bool inside = col < ncols && frame_column(fr, p.nx, p.ny, col, &i, &j);
    double hh = 0.0;
    if (inside) {
        auto fo = [&](int c) -> const float* { return fptr(p, par, c); };
        auto fn = [&](int c) -> float* { return fptr(p, par ^ 1, c); };  // E^{n+1} is here
        const bool per = p.periodic != 0;
        const int kp = k + 1 == p.nz ? 0 : k + 1;
        int ip = i + 1, jp = j + 1;
        const bool has_ip = ip < p.nx || per, has_jp = jp < p.ny || per;
        if (ip >= p.nx) ip -= p.nx;
        if (jp >= p.ny) jp -= p.ny;
        const size_t row = ((size_t)k * p.ny + j) * p.pitch;
        const size_t row_jp = ((size_t)k * p.ny + jp) * p.pitch;
        const size_t row_kp = ((size_t)kp * p.ny + j) * p.pitch;
        const size_t id = row + i;
        ENbr e;
        e.ex = fn(EX)[id];
        e.ey = fn(EY)[id];
        e.ez = fn(EZ)[id];
        e.ey_ip = has_ip ? fn(EY)[row + ip] : 0.f;
        e.ez_ip = has_ip ? fn(EZ)[row + ip] : 0.f;
        e.ex_jp = has_jp ? fn(EX)[row_jp + i] : 0.f;
        e.ez_jp = has_jp ? fn(EZ)[row_jp + i] : 0.f;
        e.ex_kp = fn(EX)[row_kp + i];
        e.ey_kp = fn(EY)[row_kp + i];
        const float hx0 = fo(HX)[id], hy0 = fo(HY)[id], hz0 = fo(HZ)[id];
        float hx = hx0, hy = hy0, hz = hz0;
        const int slot = p.colmap ? p.colmap[(size_t)j * p.nx + i] : -1;
        float2 qt0 = make_float2(0.f, 0.f), qt1 = qt0;
        if (slot >= 0) {
            const float2 t = p.tH[n];
            qt0 = cmul(p.zph[2 * k], t);
            qt1 = cmul(p.zph[2 * k + 1], t);
        }
        h_cell(p, par, i, j, k, e, hx, hy, hz, slot, qt0, qt1);
        fn(HX)[id] = hx;
        fn(HY)[id] = hy;
        fn(HZ)[id] = hz;
        hh = (double)hx0 * hx + (double)hy0 * hy + (double)hz0 * hz;
    }
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
    hipLaunchKernelGGL(split_e_kernel, grid, dim3(BT), 0, s, p, n, parity, fr, nc, epart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timer) timer->mark(fr.x1 > 0 ? "frame_h" : "split_h");
    hipLaunchKernelGGL(split_h_kernel, grid, dim3(BT), 0, s, p, n, parity, fr, nc,
                       epart ? epart + nb : nullptr);
    if (timer) timer->mark(nullptr);
    return hipGetLastError();
}

}  // namespace bfdtd
