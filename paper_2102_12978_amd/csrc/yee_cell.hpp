// Per-cell Yee updates with every boundary case (PEC walls, CPML slabs,
// periodic test mode) and the antenna soft source. Shared by the split
// kernels and the batched kernels so both compute bit-identical values for
// a cell.
#pragma once

#include "kernels_common.hpp"

namespace bfdtd {

// E update of cell (i, j, k) (paper §4 Yee scheme + CPML + soft source):
//   E_x += S_y [Δ_y H_z]_cpml - S_z Δ_z H_y
//   E_y += S_z Δ_z H_x - S_x [Δ_x H_z]_cpml
//   E_z += S_x [Δ_x H_y]_cpml - S_y [Δ_y H_x]_cpml
// with backward differences of H̃^{n+1/2}; [Δ]_cpml = Δ/κ + ψ, ψ ← b ψ + c Δ
// (ψ of the old parity read, of the new parity written when store_psi).
// E on the x = 0 / y = 0 PEC wall is held. pt0 / pt1: e^{iβz} T_E(n) at the
// integer / half z planes of this k.
struct HNbr {
    float hx, hx_jm, hx_km;    // H_x at (i, j), (i, j-1), plane k-1
    float hy, hy_im, hy_km;    // H_y at (i, j), (i-1, j), plane k-1
    float hz, hz_im, hz_jm;    // H_z at (i, j), (i-1, j), (i, j-1)
};

// BND = false compiles the wall and CPML handling out (cells known to be
// away from both).
template <bool BND = true>
__device__ __forceinline__ void e_cell(const Problem& p, int par, int i, int j, int k,
                                       const HNbr& h, float& ex, float& ey, float& ez, int slot,
                                       float2 pt0, float2 pt1, bool store_psi) {
    const bool per = p.periodic != 0;
    const float d_yhz = h.hz - h.hz_jm, d_zhy = h.hy - h.hy_km;
    const float d_zhx = h.hx - h.hx_km, d_xhz = h.hz - h.hz_im;
    const float d_xhy = h.hy - h.hy_im, d_yhx = h.hx - h.hx_jm;
    const bool hold_x = BND && !per && i == 0;   // E_y, E_z on the x = 0 wall
    const bool hold_y = BND && !per && j == 0;   // E_x, E_z on the y = 0 wall
    const int xs = BND ? slab_index(i, p.nx, p.npml) : -1;
    const int ys = BND ? slab_index(j, p.ny, p.npml) : -1;
    float tx_hz = d_xhz, tx_hy = d_xhy, ty_hz = d_yhz, ty_hx = d_yhx;
    if (xs >= 0) {
        const float b = cx_tab(p, T_EB)[i], c = cx_tab(p, T_EC)[i], kinv = cx_tab(p, T_EK)[i];
        const size_t q = psix_at(p, k, j, xs);
        float py = pptr(p, par, P_EYX)[q], pz = pptr(p, par, P_EZX)[q];
        if (!hold_x) py = cpml_mem(b, py, c, d_xhz);
        if (!hold_x && !hold_y) pz = cpml_mem(b, pz, c, d_xhy);
        if (store_psi) {
            pptr(p, par ^ 1, P_EYX)[q] = py;
            pptr(p, par ^ 1, P_EZX)[q] = pz;
        }
        tx_hz = stretched(kinv, d_xhz, py);
        tx_hy = stretched(kinv, d_xhy, pz);
    }
    if (ys >= 0) {
        const float b = cy_tab(p, T_EB)[j], c = cy_tab(p, T_EC)[j], kinv = cy_tab(p, T_EK)[j];
        const size_t q = psiy_at(p, k, ys, i);
        float px = pptr(p, par, P_EXY)[q], pz = pptr(p, par, P_EZY)[q];
        if (!hold_y) px = cpml_mem(b, px, c, d_yhz);
        if (!hold_y && !hold_x) pz = cpml_mem(b, pz, c, d_yhx);
        if (store_psi) {
            pptr(p, par ^ 1, P_EXY)[q] = px;
            pptr(p, par ^ 1, P_EZY)[q] = pz;
        }
        ty_hz = stretched(kinv, d_yhz, px);
        ty_hx = stretched(kinv, d_yhx, pz);
    }
    if (!hold_y) ex += curl_pair(p.sy, ty_hz, p.sz, d_zhy);
    if (!hold_x) ey += curl_pair(p.sz, d_zhx, p.sx, tx_hz);
    if (!hold_x && !hold_y) ez += curl_pair(p.sx, tx_hy, p.sy, ty_hx);
    if (slot >= 0) {
        const gptr<const float2> a = G(p.amp) + (size_t)slot * 6;
        ex += cmul_re(ld2(a, EX), pt0);
        ey += cmul_re(ld2(a, EY), pt0);
        ez += cmul_re(ld2(a, EZ), pt1);
    }
}

// H update of cell (i, j, k):
//   H_x -= S_y [Δ_y E_z]_cpml - S_z Δ_z E_y
//   H_y -= S_z Δ_z E_x - S_x [Δ_x E_z]_cpml
//   H_z -= S_x [Δ_x E_y]_cpml - S_y [Δ_y E_x]_cpml
// with forward differences of E^{n+1}; qt0 / qt1: e^{iβz} T_H(n).
struct ENbr {
    float ex, ex_jp, ex_kp;    // E_x at (i, j), (i, j+1), plane k+1
    float ey, ey_ip, ey_kp;    // E_y at (i, j), (i+1, j), plane k+1
    float ez, ez_ip, ez_jp;    // E_z at (i, j), (i+1, j), (i, j+1)
};

template <bool BND = true>
__device__ __forceinline__ void h_cell(const Problem& p, int par, int i, int j, int k,
                                       const ENbr& e, float& hx, float& hy, float& hz, int slot,
                                       float2 qt0, float2 qt1) {
    const float d_yez = e.ez_jp - e.ez, d_zey = e.ey_kp - e.ey;
    const float d_zex = e.ex_kp - e.ex, d_xez = e.ez_ip - e.ez;
    const float d_xey = e.ey_ip - e.ey, d_yex = e.ex_jp - e.ex;
    const int xs = BND ? slab_index(i, p.nx, p.npml) : -1;
    const int ys = BND ? slab_index(j, p.ny, p.npml) : -1;
    float tx_ez = d_xez, tx_ey = d_xey, ty_ez = d_yez, ty_ex = d_yex;
    if (xs >= 0) {
        const float b = cx_tab(p, T_HB)[i], c = cx_tab(p, T_HC)[i], kinv = cx_tab(p, T_HK)[i];
        const size_t q = psix_at(p, k, j, xs);
        const float py = cpml_mem(b, pptr(p, par, P_HYX)[q], c, d_xez);
        const float pz = cpml_mem(b, pptr(p, par, P_HZX)[q], c, d_xey);
        pptr(p, par ^ 1, P_HYX)[q] = py;
        pptr(p, par ^ 1, P_HZX)[q] = pz;
        tx_ez = stretched(kinv, d_xez, py);
        tx_ey = stretched(kinv, d_xey, pz);
    }
    if (ys >= 0) {
        const float b = cy_tab(p, T_HB)[j], c = cy_tab(p, T_HC)[j], kinv = cy_tab(p, T_HK)[j];
        const size_t q = psiy_at(p, k, ys, i);
        const float px = cpml_mem(b, pptr(p, par, P_HXY)[q], c, d_yez);
        const float pz = cpml_mem(b, pptr(p, par, P_HZY)[q], c, d_yex);
        pptr(p, par ^ 1, P_HXY)[q] = px;
        pptr(p, par ^ 1, P_HZY)[q] = pz;
        ty_ez = stretched(kinv, d_yez, px);
        ty_ex = stretched(kinv, d_yex, pz);
    }
    hx -= curl_pair(p.sy, ty_ez, p.sz, d_zey);
    hy -= curl_pair(p.sz, d_zex, p.sx, tx_ez);
    hz -= curl_pair(p.sx, tx_ey, p.sy, ty_ex);
    if (slot >= 0) {
        const gptr<const float2> a = G(p.amp) + (size_t)slot * 6;
        hx += cmul_re(ld2(a, HX), qt1);
        hy += cmul_re(ld2(a, HY), qt1);
        hz += cmul_re(ld2(a, HZ), qt0);
    }
}

// E update of cell (i, j, k) of parity par -> par ^ 1 with its neighbour
// loads, the E source at step n and the plane accumulation selected by
// diag_mask. Returns |E^{n+1}|² at the cell (for the energy).
__device__ __forceinline__ double e_point(const Problem& p, long long n, int par, int i, int j,
                                          int k, int diag_mask) {
    auto fo = [&](int c) { return fptr(p, par, c); };
    auto fn = [&](int c) { return fptr(p, par ^ 1, c); };
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
    const int slot = p.colmap ? G(p.colmap)[(size_t)j * p.nx + i] : -1;
    float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
    if (slot >= 0) {
        const float2 t = ldc2(p.tE, n);
        pt0 = cmul(ldc2(p.zph, 2 * k), t);
        pt1 = cmul(ldc2(p.zph, 2 * k + 1), t);
    }
    e_cell(p, par, i, j, k, h, ex, ey, ez, slot, pt0, pt1, true);
    fn(EX)[id] = ex;
    fn(EY)[id] = ey;
    fn(EZ)[id] = ez;
    if (k == p.plane && diag_mask) {
        const size_t pl = (size_t)j * p.nx + i, ps = (size_t)p.nx * p.ny;
        const gptr<double> fl = G(p.fl);
        if (diag_mask & FDTD_DIAG_EX2) fl[pl] = sq_acc(fl[pl], ex);
        if (diag_mask & FDTD_DIAG_EY2) fl[ps + pl] = sq_acc(fl[ps + pl], ey);
        if (diag_mask & FDTD_DIAG_EZ2) fl[2 * ps + pl] = sq_acc(fl[2 * ps + pl], ez);
    }
    if (k == p.plane && p.rec) G(p.rec)[(size_t)(n - p.rec_begin) * p.nx * p.ny + (size_t)j * p.nx + i] = ey;
    return (double)ex * ex + (double)ey * ey + (double)ez * ez;
}

// H update of cell (i, j, k): H of parity par and E^{n+1} of parity par ^ 1
// -> H of parity par ^ 1, with the H source at step n. Returns
// H^{n+1/2}·H^{n+3/2} at the cell (for the energy).
__device__ __forceinline__ double h_point(const Problem& p, long long n, int par, int i, int j,
                                          int k) {
    auto fo = [&](int c) { return fptr(p, par, c); };
    auto fn = [&](int c) { return fptr(p, par ^ 1, c); };   // E^{n+1} is here
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
    const int slot = p.colmap ? G(p.colmap)[(size_t)j * p.nx + i] : -1;
    float2 qt0 = make_float2(0.f, 0.f), qt1 = qt0;
    if (slot >= 0) {
        const float2 t = ldc2(p.tH, n);
        qt0 = cmul(ldc2(p.zph, 2 * k), t);
        qt1 = cmul(ldc2(p.zph, 2 * k + 1), t);
    }
    h_cell(p, par, i, j, k, e, hx, hy, hz, slot, qt0, qt1);
    fn(HX)[id] = hx;
    fn(HY)[id] = hy;
    fn(HZ)[id] = hz;
    return (double)hx0 * hx + (double)hy0 * hy + (double)hz0 * hz;
}

}  // namespace bfdtd
