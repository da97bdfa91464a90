// Transposed Yee step (reverse-mode differentiation of the linear scheme).
//
// The forward step maps x = (E, H̃, ψ_E, ψ_H) to F x + s(t) with the antenna
// source s independent of x. Its transpose is taken term by term. For a curl
// term of the forward update
//     ψ' = b ψ + c Δ,   u' = u + σ S_d ((1/κ) Δ + ψ'),   Δ = D v
// (D a backward difference for the E part, a forward one for the H part,
// b = c = 0 and 1/κ = 1 outside the CPML slabs), the transpose with
// adjoint variables λ reads
//     μ = σ S_d λ_u',   λ_Δ = (1/κ + c) μ + c λ_ψ',   λ_ψ = b (μ + λ_ψ'),
//     λ_u = λ_u',       λ_v += Dᵀ λ_Δ = -D_f λ_Δ (E part) or -D_b λ_Δ (H part).
// E components held by the PEC walls are not updated forward, so their μ is
// zero and their λ_ψ passes through unchanged.
//
// The reverse step undoes the H part first, then the E part. λ is
// ping-ponged like the forward fields: the H-part transpose forms λ_E of
// parity par ^ 1 from λ_E and λ_H of parity par, the E-part transpose forms
// λ_H of parity par ^ 1 from λ_H of parity par and the new λ_E; the new λ_ψ
// go to parity par ^ 1 as well. On cells away from walls and CPML this is
// the forward Yee step with S_x, S_y, S_z negated and no source, which the
// fused interior kernel runs (adjoint.cpp); these kernels take the frame
// around that interior (or the whole grid). One thread per cell; grid
// (frame columns / 256, nz).
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int BT = 256;

// vpar: parity of the other family's λ that the update reads (par for the
// H-part transpose, par ^ 1, the new λ_E, for the E-part transpose).
struct Lam {
    const Problem& p;
    int par, vpar, i, j, k;
    __device__ gptr<const float> fo(int c) const {   // own family, parity par
        return G((const float*)p.fbase[par]) + c * p.fstride;
    }
    __device__ gptr<float> fn(int c) const {         // own family, parity par ^ 1
        return G(p.fbase[par ^ 1]) + c * p.fstride;
    }
    __device__ size_t at(int ii, int jj, int kk) const {
        return ((size_t)kk * p.ny + jj) * p.pitch + ii;
    }
    __device__ float v(int c, int ii, int jj, int kk) const {
        return (G((const float*)p.fbase[vpar]) + c * p.fstride)[at(ii, jj, kk)];
    }
    __device__ gptr<const float> psi_old(int q) const { return pptr(p, par, q); }
    __device__ gptr<float> psi_new(int q) const { return pptr(p, par ^ 1, q); }
};

// ---- H part transposed: λ_E += -D_b λ_Δ of the H terms ------------------
// λ_Δ of the H term (h_comp, d = x) at column ii of row j, plane k.
__device__ __forceinline__ float dh_x(const Lam& L, int hc, int q, float sign, int ii) {
    const Problem& p = L.p;
    if (ii < 0) {
        if (!p.periodic) return 0.f;
        ii += p.nx;
    }
    const float mu = sign * p.sx * L.v(hc, ii, L.j, L.k);
    const int xs = slab_index(ii, p.nx, p.npml);
    if (xs < 0) return mu;
    const float c = cx_tab(p, T_HC)[ii], kinv = cx_tab(p, T_HK)[ii];
    return (kinv + c) * mu + c * L.psi_old(q)[psix_at(p, L.k, L.j, xs)];
}

__device__ __forceinline__ float dh_y(const Lam& L, int hc, int q, float sign, int jj) {
    const Problem& p = L.p;
    if (jj < 0) {
        if (!p.periodic) return 0.f;
        jj += p.ny;
    }
    const float mu = sign * p.sy * L.v(hc, L.i, jj, L.k);
    const int ys = slab_index(jj, p.ny, p.npml);
    if (ys < 0) return mu;
    const float c = cy_tab(p, T_HC)[jj], kinv = cy_tab(p, T_HK)[jj];
    return (kinv + c) * mu + c * L.psi_old(q)[psiy_at(p, L.k, ys, L.i)];
}

__device__ __forceinline__ float dh_z(const Lam& L, int hc, float sign, int kk) {
    const Problem& p = L.p;
    if (kk < 0) kk += p.nz;
    return sign * p.sz * L.v(hc, L.i, L.j, kk);
}

__global__ void __launch_bounds__(BT) adj_h_kernel(Problem p, int par, Frame fr, long long ncols) {
    int ci = 0, cj = 0;
    const unsigned col = blockIdx.x * BT + threadIdx.x;
    if (col >= (unsigned long long)ncols || !frame_column(fr, p.nx, p.ny, col, &ci, &cj)) return;
    const Lam L{p, par, par, ci, cj, (int)blockIdx.y};
    const int i = L.i, j = L.j, k = L.k;
    const size_t id = L.at(i, j, k);
    // H terms: hx: (ez, y, -1, ψ_hxy) (ey, z, +1); hy: (ex, z, -1) (ez, x, +1, ψ_hyx);
    //          hz: (ey, x, -1, ψ_hzx) (ex, y, +1, ψ_hzy)
    const float gx = -(dh_z(L, HY, -1.f, k) - dh_z(L, HY, -1.f, k - 1)) -
                     (dh_y(L, HZ, P_HZY, 1.f, j) - dh_y(L, HZ, P_HZY, 1.f, j - 1));
    const float gy = -(dh_z(L, HX, 1.f, k) - dh_z(L, HX, 1.f, k - 1)) -
                     (dh_x(L, HZ, P_HZX, -1.f, i) - dh_x(L, HZ, P_HZX, -1.f, i - 1));
    const float gz = -(dh_y(L, HX, P_HXY, -1.f, j) - dh_y(L, HX, P_HXY, -1.f, j - 1)) -
                     (dh_x(L, HY, P_HYX, 1.f, i) - dh_x(L, HY, P_HYX, 1.f, i - 1));
    const float ox = L.fo(EX)[id], oy = L.fo(EY)[id], oz = L.fo(EZ)[id];
    // λ_ψ of the H memories at this cell. Every load comes before the first
    // store: the compiler cannot tell the buffers apart, and a load after a
    // store would wait for it.
    const int xs = slab_index(i, p.nx, p.npml), ys = slab_index(j, p.ny, p.npml);
    float yx = 0.f, zx = 0.f, xy = 0.f, zy = 0.f;
    size_t qx = 0, qy = 0;
    if (xs >= 0) {
        const float b = cx_tab(p, T_HB)[i];
        qx = psix_at(p, k, j, xs);
        yx = b * (p.sx * L.v(HY, i, j, k) + L.psi_old(P_HYX)[qx]);
        zx = b * (-p.sx * L.v(HZ, i, j, k) + L.psi_old(P_HZX)[qx]);
    }
    if (ys >= 0) {
        const float b = cy_tab(p, T_HB)[j];
        qy = psiy_at(p, k, ys, i);
        xy = b * (-p.sy * L.v(HX, i, j, k) + L.psi_old(P_HXY)[qy]);
        zy = b * (p.sy * L.v(HZ, i, j, k) + L.psi_old(P_HZY)[qy]);
    }
    L.fn(EX)[id] = ox + gx;
    L.fn(EY)[id] = oy + gy;
    L.fn(EZ)[id] = oz + gz;
    if (xs >= 0) {
        L.psi_new(P_HYX)[qx] = yx;
        L.psi_new(P_HZX)[qx] = zx;
    }
    if (ys >= 0) {
        L.psi_new(P_HXY)[qy] = xy;
        L.psi_new(P_HZY)[qy] = zy;
    }
}

// ---- E part transposed: λ_H += -D_f λ_Δ of the E terms ------------------
// E components updated at (ii, jj): E_y and E_z are held on the x = 0 wall,
// E_x and E_z on the y = 0 wall.
__device__ __forceinline__ bool upd_e(const Problem& p, int ec, int ii, int jj) {
    if (p.periodic) return true;
    const bool hx = ii == 0, hy = jj == 0;
    if (ec == EX) return !hy;
    if (ec == EY) return !hx;
    return !hx && !hy;
}

__device__ __forceinline__ float de_x(const Lam& L, int ec, int q, float sign, int ii) {
    const Problem& p = L.p;
    if (ii >= p.nx) {
        if (!p.periodic) return 0.f;
        ii -= p.nx;
    }
    if (!upd_e(p, ec, ii, L.j)) return 0.f;
    const float mu = sign * p.sx * L.v(ec, ii, L.j, L.k);
    const int xs = slab_index(ii, p.nx, p.npml);
    if (xs < 0) return mu;
    const float c = cx_tab(p, T_EC)[ii], kinv = cx_tab(p, T_EK)[ii];
    return (kinv + c) * mu + c * L.psi_old(q)[psix_at(p, L.k, L.j, xs)];
}

__device__ __forceinline__ float de_y(const Lam& L, int ec, int q, float sign, int jj) {
    const Problem& p = L.p;
    if (jj >= p.ny) {
        if (!p.periodic) return 0.f;
        jj -= p.ny;
    }
    if (!upd_e(p, ec, L.i, jj)) return 0.f;
    const float mu = sign * p.sy * L.v(ec, L.i, jj, L.k);
    const int ys = slab_index(jj, p.ny, p.npml);
    if (ys < 0) return mu;
    const float c = cy_tab(p, T_EC)[jj], kinv = cy_tab(p, T_EK)[jj];
    return (kinv + c) * mu + c * L.psi_old(q)[psiy_at(p, L.k, ys, L.i)];
}

__device__ __forceinline__ float de_z(const Lam& L, int ec, float sign, int kk) {
    const Problem& p = L.p;
    if (kk >= p.nz) kk -= p.nz;
    if (!upd_e(p, ec, L.i, L.j)) return 0.f;
    return sign * p.sz * L.v(ec, L.i, L.j, kk);
}

__global__ void __launch_bounds__(BT) adj_e_kernel(Problem p, int par, Frame fr, long long ncols) {
    int ci = 0, cj = 0;
    const unsigned col = blockIdx.x * BT + threadIdx.x;
    if (col >= (unsigned long long)ncols || !frame_column(fr, p.nx, p.ny, col, &ci, &cj)) return;
    const Lam L{p, par, par ^ 1, ci, cj, (int)blockIdx.y};
    const int i = L.i, j = L.j, k = L.k;
    const size_t id = L.at(i, j, k);
    // E terms: ex: (hz, y, +1, ψ_exy) (hy, z, -1); ey: (hx, z, +1) (hz, x, -1, ψ_eyx);
    //          ez: (hy, x, +1, ψ_ezx) (hx, y, -1, ψ_ezy)
    const float gx = -(de_z(L, EY, 1.f, k + 1) - de_z(L, EY, 1.f, k)) -
                     (de_y(L, EZ, P_EZY, -1.f, j + 1) - de_y(L, EZ, P_EZY, -1.f, j));
    const float gy = -(de_z(L, EX, -1.f, k + 1) - de_z(L, EX, -1.f, k)) -
                     (de_x(L, EZ, P_EZX, 1.f, i + 1) - de_x(L, EZ, P_EZX, 1.f, i));
    const float gz = -(de_y(L, EX, P_EXY, 1.f, j + 1) - de_y(L, EX, P_EXY, 1.f, j)) -
                     (de_x(L, EY, P_EYX, -1.f, i + 1) - de_x(L, EY, P_EYX, -1.f, i));
    const float ox = L.fo(HX)[id], oy = L.fo(HY)[id], oz = L.fo(HZ)[id];
    // every load before the first store, as in adj_h_kernel
    const int xs = slab_index(i, p.nx, p.npml), ys = slab_index(j, p.ny, p.npml);
    float yx = 0.f, zx = 0.f, xy = 0.f, zy = 0.f;
    size_t qx = 0, qy = 0;
    if (xs >= 0) {
        const float b = cx_tab(p, T_EB)[i];
        qx = psix_at(p, k, j, xs);
        const float py = L.psi_old(P_EYX)[qx], pz = L.psi_old(P_EZX)[qx];
        yx = upd_e(p, EY, i, j) ? b * (-p.sx * L.v(EY, i, j, k) + py) : py;
        zx = upd_e(p, EZ, i, j) ? b * (p.sx * L.v(EZ, i, j, k) + pz) : pz;
    }
    if (ys >= 0) {
        const float b = cy_tab(p, T_EB)[j];
        qy = psiy_at(p, k, ys, i);
        const float px = L.psi_old(P_EXY)[qy], pz = L.psi_old(P_EZY)[qy];
        xy = upd_e(p, EX, i, j) ? b * (p.sy * L.v(EX, i, j, k) + px) : px;
        zy = upd_e(p, EZ, i, j) ? b * (-p.sy * L.v(EZ, i, j, k) + pz) : pz;
    }
    L.fn(HX)[id] = ox + gx;
    L.fn(HY)[id] = oy + gy;
    L.fn(HZ)[id] = oz + gz;
    if (xs >= 0) {
        L.psi_new(P_EYX)[qx] = yx;
        L.psi_new(P_EZX)[qx] = zx;
    }
    if (ys >= 0) {
        L.psi_new(P_EXY)[qy] = xy;
        L.psi_new(P_EZY)[qy] = zy;
    }
}

// ∂L/∂E_y^{n+1} on the intensity plane: λ_Ey += coef · g · E_y (the
// intensity is the window mean of E_y², g = ∂L/∂Ī).
__global__ void __launch_bounds__(BT) adj_inject_kernel(Problem p, int par, const float* g,
                                                        const float* ey, float coef) {
    const int col = blockIdx.x * BT + threadIdx.x;
    if (col >= p.nx * p.ny) return;
    const int i = col % p.nx, j = col / p.nx;
    const gptr<float> f = G(p.fbase[par]) + EY * p.fstride;
    f[((size_t)p.plane * p.ny + j) * p.pitch + i] += coef * g[col] * ey[col];
}

// G_c(slot) += T(t) Σ_k λ_c(k, j, i) e^{iβ z_c(k)} for one step: the six
// components of every antenna column, in double; the H components read λ
// of parity par_h at the H time factor tH, the E components λ of parity
// par_e at tE.
// One wavefront per (antenna column, component): lane l sums the planes
// k = l, l + 64, ... of that column, then the wavefront adds the lanes in a
// fixed butterfly order, so the result does not depend on scheduling. All
// planes of a column are in flight at once (a thread per column would walk
// them one after another).
__global__ void __launch_bounds__(BT) adj_gacc_kernel(Problem p, int par_h, int par_e,
                                                      const int* slot_i, const int* slot_j,
                                                      int nslots, float2 tH, float2 tE,
                                                      double2* G) {
    const int pair = blockIdx.x * (BT / 64) + (int)(threadIdx.x >> 6);
    if (pair >= nslots * 6) return;                      // whole wavefront
    const int lane = threadIdx.x & 63;
    const int s = pair / 6, c = pair % 6;
    const bool is_e = c <= EZ;
    const int par = is_e ? par_e : par_h;
    const float2 t = is_e ? tE : tH;
    const int i = slot_i[s], j = slot_j[s];
    // integer-plane components: E_x, E_y, H_z; half-plane: E_z, H_x, H_y
    const int half = (c == EZ || c == HX || c == HY) ? 1 : 0;
    const float* f = p.fbase[par] + c * p.fstride + (size_t)j * p.pitch + i;
    const size_t plane = (size_t)p.ny * p.pitch;
    double re = 0.0, im = 0.0;
    for (int k = lane; k < p.nz; k += 64) {
        const double l = f[k * plane];
        const float2 z = p.zph[2 * k + half];
        re += l * z.x;
        im += l * z.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        double2 g = G[(size_t)s * 6 + c];
        g.x += re * t.x - im * t.y;
        g.y += re * t.y + im * t.x;
        G[(size_t)s * 6 + c] = g;
    }
}

}  // namespace

hipError_t launch_adjoint_h(const Problem& lam, int par, const Frame& fr, hipStream_t s) {
    const long long nc = frame_columns(lam, fr);
    if (nc == 0) return hipSuccess;
    dim3 grid((unsigned)((nc + BT - 1) / BT), lam.nz);
    hipLaunchKernelGGL(adj_h_kernel, grid, dim3(BT), 0, s, lam, par, fr, nc);
    return hipGetLastError();
}

hipError_t launch_adjoint_e(const Problem& lam, int par, const Frame& fr, hipStream_t s) {
    const long long nc = frame_columns(lam, fr);
    if (nc == 0) return hipSuccess;
    dim3 grid((unsigned)((nc + BT - 1) / BT), lam.nz);
    hipLaunchKernelGGL(adj_e_kernel, grid, dim3(BT), 0, s, lam, par, fr, nc);
    return hipGetLastError();
}

hipError_t launch_adjoint_inject(const Problem& lam, int par, const float* g, const float* ey,
                                 float coef, hipStream_t s) {
    hipLaunchKernelGGL(adj_inject_kernel, dim3((lam.nx * lam.ny + BT - 1) / BT), dim3(BT), 0, s,
                       lam, par, g, ey, coef);
    return hipGetLastError();
}

hipError_t launch_adjoint_gacc(const Problem& lam, int par_h, int par_e, const int* slot_i,
                               const int* slot_j, int nslots, float2 tH, float2 tE, double2* G,
                               hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const int waves = BT / 64;
    hipLaunchKernelGGL(adj_gacc_kernel, dim3((nslots * 6 + waves - 1) / waves), dim3(BT), 0, s,
                       lam, par_h, par_e, slot_i, slot_j, nslots, tH, tE, G);
    return hipGetLastError();
}

}  // namespace bfdtd
