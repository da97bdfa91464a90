// Two-kernel Yee step (one thread per cell): E update + E source, then
// H update + H source, each reading the old ping-pong buffer and writing the
// new one. It carries every boundary case (PEC walls, CPML slabs, periodic
// wrap) and moves 72 B per cell-update.
//
// It runs either on the whole grid (FDTD_KERNEL_SPLIT) or on the frame of
// cells around the interior rectangle that the fused kernel handles; the
// frame is enumerated as a flat list of (x, y) columns: the bottom rows
// y < y0, the top rows y >= y1, then the left (x < x0) and right (x >= x1)
// strips of the rows in between.
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"

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
        const float hx = fo(HX)[id], hy = fo(HY)[id], hz = fo(HZ)[id];
        const float hz_im = has_im ? fo(HZ)[row + im] : 0.f;
        const float hy_im = has_im ? fo(HY)[row + im] : 0.f;
        const float hz_jm = has_jm ? fo(HZ)[row_jm + i] : 0.f;
        const float hx_jm = has_jm ? fo(HX)[row_jm + i] : 0.f;
        const float hy_km = fo(HY)[row_km + i];
        const float hx_km = fo(HX)[row_km + i];
        const float d_yhz = hz - hz_jm, d_zhy = hy - hy_km;
        const float d_zhx = hx - hx_km, d_xhz = hz - hz_im;
        const float d_xhy = hy - hy_im, d_yhx = hx - hx_jm;

        float ex = fo(EX)[id], ey = fo(EY)[id], ez = fo(EZ)[id];
        const bool hold_x = !per && i == 0;   // E_y, E_z on the x = 0 wall
        const bool hold_y = !per && j == 0;   // E_x, E_z on the y = 0 wall
        const int xs = slab_index(i, p.nx, p.npml);
        const int ys = slab_index(j, p.ny, p.npml);

        float tx_hz = d_xhz, tx_hy = d_xhy, ty_hz = d_yhz, ty_hx = d_yhx;
        if (xs >= 0) {
            const float b = cx_tab(p, T_EB)[i], c = cx_tab(p, T_EC)[i], kinv = cx_tab(p, T_EK)[i];
            const size_t q = psix_at(p, k, j, xs);
            float py = pptr(p, par, P_EYX)[q], pz = pptr(p, par, P_EZX)[q];
            if (!hold_x) py = b * py + c * d_xhz;
            if (!hold_x && !hold_y) pz = b * pz + c * d_xhy;
            pptr(p, par ^ 1, P_EYX)[q] = py;
            pptr(p, par ^ 1, P_EZX)[q] = pz;
            tx_hz = kinv * d_xhz + py;
            tx_hy = kinv * d_xhy + pz;
        }
        if (ys >= 0) {
            const float b = cy_tab(p, T_EB)[j], c = cy_tab(p, T_EC)[j], kinv = cy_tab(p, T_EK)[j];
            const size_t q = psiy_at(p, k, ys, i);
            float px = pptr(p, par, P_EXY)[q], pz = pptr(p, par, P_EZY)[q];
            if (!hold_y) px = b * px + c * d_yhz;
            if (!hold_y && !hold_x) pz = b * pz + c * d_yhx;
            pptr(p, par ^ 1, P_EXY)[q] = px;
            pptr(p, par ^ 1, P_EZY)[q] = pz;
            ty_hz = kinv * d_yhz + px;
            ty_hx = kinv * d_yhx + pz;
        }
        if (!hold_y) ex += p.sy * ty_hz - p.sz * d_zhy;
        if (!hold_x) ey += p.sz * d_zhx - p.sx * tx_hz;
        if (!hold_x && !hold_y) ez += p.sx * tx_hy - p.sy * ty_hx;
        if (p.colmap) {
            const int slot = p.colmap[(size_t)j * p.nx + i];
            if (slot >= 0) {
                const float2 t = p.tE[n];
                const float2 pi0 = cmul(p.zph[2 * k], t), pi1 = cmul(p.zph[2 * k + 1], t);
                const float2* a = p.amp + (size_t)slot * 6;
                ex += cmul_re(a[EX], pi0);
                ey += cmul_re(a[EY], pi0);
                ez += cmul_re(a[EZ], pi1);
            }
        }
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
        const float ex = fn(EX)[id], ey = fn(EY)[id], ez = fn(EZ)[id];
        const float ey_ip = has_ip ? fn(EY)[row + ip] : 0.f;
        const float ez_ip = has_ip ? fn(EZ)[row + ip] : 0.f;
        const float ex_jp = has_jp ? fn(EX)[row_jp + i] : 0.f;
        const float ez_jp = has_jp ? fn(EZ)[row_jp + i] : 0.f;
        const float ex_kp = fn(EX)[row_kp + i];
        const float ey_kp = fn(EY)[row_kp + i];
        const float d_yez = ez_jp - ez, d_zey = ey_kp - ey;
        const float d_zex = ex_kp - ex, d_xez = ez_ip - ez;
        const float d_xey = ey_ip - ey, d_yex = ex_jp - ex;

        const float hx0 = fo(HX)[id], hy0 = fo(HY)[id], hz0 = fo(HZ)[id];
        const int xs = slab_index(i, p.nx, p.npml);
        const int ys = slab_index(j, p.ny, p.npml);
        float tx_ez = d_xez, tx_ey = d_xey, ty_ez = d_yez, ty_ex = d_yex;
        if (xs >= 0) {
            const float b = cx_tab(p, T_HB)[i], c = cx_tab(p, T_HC)[i], kinv = cx_tab(p, T_HK)[i];
            const size_t q = psix_at(p, k, j, xs);
            const float py = b * pptr(p, par, P_HYX)[q] + c * d_xez;
            const float pz = b * pptr(p, par, P_HZX)[q] + c * d_xey;
            pptr(p, par ^ 1, P_HYX)[q] = py;
            pptr(p, par ^ 1, P_HZX)[q] = pz;
            tx_ez = kinv * d_xez + py;
            tx_ey = kinv * d_xey + pz;
        }
        if (ys >= 0) {
            const float b = cy_tab(p, T_HB)[j], c = cy_tab(p, T_HC)[j], kinv = cy_tab(p, T_HK)[j];
            const size_t q = psiy_at(p, k, ys, i);
            const float px = b * pptr(p, par, P_HXY)[q] + c * d_yez;
            const float pz = b * pptr(p, par, P_HZY)[q] + c * d_yex;
            pptr(p, par ^ 1, P_HXY)[q] = px;
            pptr(p, par ^ 1, P_HZY)[q] = pz;
            ty_ez = kinv * d_yez + px;
            ty_ex = kinv * d_yex + pz;
        }
        float hx = hx0 - (p.sy * ty_ez - p.sz * d_zey);
        float hy = hy0 - (p.sz * d_zex - p.sx * tx_ez);
        float hz = hz0 - (p.sx * tx_ey - p.sy * ty_ex);
        if (p.colmap) {
            const int slot = p.colmap[(size_t)j * p.nx + i];
            if (slot >= 0) {
                const float2 t = p.tH[n];
                const float2 pi0 = cmul(p.zph[2 * k], t), pi1 = cmul(p.zph[2 * k + 1], t);
                const float2* a = p.amp + (size_t)slot * 6;
                hx += cmul_re(a[HX], pi1);
                hy += cmul_re(a[HY], pi1);
                hz += cmul_re(a[HZ], pi0);
            }
        }
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
