// Two-kernel Yee step (one thread per cell): E update + E source, then
// H update + H source, each reading the old ping-pong buffer and writing the
// new one. The plain form of the step; it moves 72 B per cell-update and
// serves as the cross-check of the fused kernel.
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ void block_energy(double v, double* out) {
    __shared__ double red[BX * BY / 64];
    v = wave_sum(v);
    int tid = threadIdx.y * BX + threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < BX * BY / 64; ++w) s += red[w];
        *out = s;
    }
}

__global__ void __launch_bounds__(BX * BY)
split_e_kernel(Problem p, long long n, int par) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool inside = i < p.nx && j < p.ny;
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
            if (!hold_y) {
                px = b * px + c * d_yhz;
            }
            if (!hold_y && !hold_x) {
                pz = b * pz + c * d_yhx;
            }
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
        if (k == p.plane && p.diag_mask) {
            const size_t pl = (size_t)j * p.nx + i, ps = (size_t)p.nx * p.ny;
            if (p.diag_mask & FDTD_DIAG_EX2) p.fl[pl] += (double)ex * ex;
            if (p.diag_mask & FDTD_DIAG_EY2) p.fl[ps + pl] += (double)ey * ey;
            if (p.diag_mask & FDTD_DIAG_EZ2) p.fl[2 * ps + pl] += (double)ez * ez;
        }
        if (p.rec && k == p.plane) p.rec[(size_t)(n - p.rec_begin) * p.nx * p.ny +
                                         (size_t)j * p.nx + i] = ey;
        e2 = (double)ex * ex + (double)ey * ey + (double)ez * ez;
    }
    if (p.epart) {
        const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_energy(e2, p.epart + b);
    }
}

__global__ void __launch_bounds__(BX * BY)
split_h_kernel(Problem p, long long n, int par) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool inside = i < p.nx && j < p.ny;
    double hh = 0.0;
    if (inside) {
        auto fo = [&](int c) -> const float* { return fptr(p, par, c); };
        auto fn = [&](int c) -> float* { return fptr(p, par ^ 1, c); };   // E^{n+1} already written here
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
    if (p.epart) {
        const size_t nb = (size_t)gridDim.x * gridDim.y * gridDim.z;
        const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_energy(hh, p.epart + nb + b);
    }
}

}  // namespace

hipError_t launch_split_step(const Problem& p, long long n, int parity, hipStream_t s) {
    dim3 block(BX, BY, 1);
    dim3 grid((p.nx + BX - 1) / BX, (p.ny + BY - 1) / BY, p.nz);
    hipLaunchKernelGGL(split_e_kernel, grid, block, 0, s, p, n, parity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_h_kernel, grid, block, 0, s, p, n, parity);
    return hipGetLastError();
}

int split_partial_count(const Problem& p) {
    return 2 * ((p.nx + BX - 1) / BX) * ((p.ny + BY - 1) / BY) * p.nz;
}

}  // namespace bfdtd
