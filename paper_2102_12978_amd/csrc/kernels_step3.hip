// Three-step Yee kernel over the whole grid (temporal blocking over three
// leapfrog steps): one pass over the fields advances every cell from E^n,
// H^{n+1/2}, CPML memories ψ^n to E^{n+3}, H^{n+7/2}, ψ^{n+3}, with the
// antenna's soft source (§4) folded in: the old ping-pong buffers are read
// once and the new ones written once, 48 B of field traffic per cell for
// three cell-updates. Each cell is formed with the expressions of the
// one-step cell code (yee_cell.hpp), in the same order, so a pass equals
// three one-step launches bit for bit.
//
// Work decomposition (CDNA4, wave64), the two-step kernel's with a third
// stage. A wavefront reads a block of 64 x cells (lane l at x = 58 s - 3 + l
// for x segment s) by TY + 6 rows (j0 - 3 .. j0 + TY + 2) and marches along
// z. Each stage is formed in registers on every lane and row it can be
// formed on, one lane and one row fewer at each side than the stage before,
// so the last stage needs nothing from other wavefronts:
//   x: neighbours move between lanes with DPP wavefront shifts; lanes 0-2
//      and 61-63 are halo and the wavefront stores lanes 3..60 (58 cells).
//   y: E^{n+1} on rows -2 .. TY+2, H^{n+3/2} on -2 .. TY+1, E^{n+2} on
//      -1 .. TY+1, H^{n+5/2} on -1 .. TY, E^{n+3} on 0 .. TY and H^{n+7/2}
//      on the TY stored rows. E_y is not formed on the last row of an E
//      stage, nor H_y on the first row of the first two H stages: nothing
//      reads them there (E_y and H_y have no y neighbour in the curls).
//   z: at plane q the pipeline forms E^{n+1}(q), H^{n+3/2}(q-1),
//      E^{n+2}(q-1), H^{n+5/2}(q-2), E^{n+3}(q-2) and H^{n+7/2}(q-3), keeping
//      one plane of each in registers; a chunk [kb, ke) reads planes
//      kb-3 .. ke+2 (z is periodic).
// Waits, as in the two-step kernel: a plane issues all its vector loads at
// its start (field rows and the CPML memories of the first stage), reads
// the z phases e^{iβz} and time factors with scalar loads (the phases of
// planes q-1 .. q-3 carried in registers) and the antenna amplitudes from
// LDS (staged once per tile), so that no stage waits for a vector load and
// with it for the plane's stores in flight. Boundary tiles load every row
// and CPML memory unconditionally (rows outside the grid read the nearest
// row inside it; lanes and rows off the slabs read slab column or row 0)
// and keep their y coefficients in LDS: a load under a branch there made
// the compiler wait for it and move it to scratch memory.
// A workgroup stacks four wavefronts in y that start every plane together
// (one barrier per plane): a row group of 4 TY rows.
//
// Tiles (segment, row group) fall in the two-step kernel's four classes,
// each its own launch and instantiation: interior (every formed cell
// regular), x boundary (per-lane CPML coefficients, held E_y/E_z at x = 0,
// zero E beyond x = nx - 1), y boundary (per-row coefficients, held
// E_x/E_z at y = 0, zero E beyond y = ny - 1) and corners. On a boundary
// lane outside the slabs the CPML form runs with b = c = 0 and 1/κ = 1,
// which gives the plain update's value exactly. Lanes and rows outside the
// grid feed only cells outside the grid or held on a wall, at every stage.
//
// The x-slab memories are [z][y][2 npml], the y-slab memories
// [z][2 npml][pitch]; a pass reads those of parity par and writes those of
// parity par ^ 1, like the fields.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int WAVES = 4;   // wavefronts per workgroup, stacked in y
constexpr int OWN = 58;    // x cells stored per wavefront (lanes 3..60)
constexpr int O = 3;       // register index of row r is r + O (rows -3 .. TY+2)

// A wave-uniform global pointer as a byte pointer held in scalar registers.
template <typename T>
__device__ __forceinline__ gptr<char> uniform3(gptr<T> q) {
    const unsigned long long a = (unsigned long long)q;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    return (gptr<char>)(((unsigned long long)hi << 32) | lo);
}

// Cross-lane moves by one lane (DPP wavefront shifts). Lanes without a
// source keep their own value.
__device__ __forceinline__ float lane_below(float v) {   // lane l gets lane l - 1
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_above(float v) {   // lane l gets lane l + 1
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x130, 0xf, 0xf, false));
}

// Indices [a0, a1) then [b0, b1).
struct Span3 {
    int a0, a1, b0, b1;
};
__host__ __device__ __forceinline__ int count3(const Span3& s) {
    return (s.a1 - s.a0) + (s.b1 - s.b0);
}
__device__ __forceinline__ int at3(const Span3& s, int i) {
    const int na = s.a1 - s.a0;
    return i < na ? s.a0 + i : s.b0 + (i - na);
}

// One launch: its x segments and row groups, the z chunks, and the cells
// segment 0 owns (xa; segment s > 0 owns the 58 from xa + 58 (s - 1)).
struct Launch3 {
    Span3 seg, grp;
    int cz, ncz, xa;
};

// x cells [lo, hi) segment s owns: segment 0 the first xa, then 58 each,
// the last one to nx.
__host__ __device__ __forceinline__ int own_lo3(int s, int xa) {
    return s == 0 ? 0 : xa + OWN * (s - 1);
}
__host__ __device__ __forceinline__ int own_hi3(int s, int xa, int nx) {
    return min(s == 0 ? xa : own_lo3(s, xa) + OWN, nx);
}

// CPML coefficients of one position: b, c and 1/κ (identity outside a slab).
struct Coef3 {
    float b, c, k;
};

// One tile: x segment seg, row group grp, planes [kb, ke) of problem p,
// advanced from step n (parity par) to n + 3; mask0..2: plane sums of
// steps n + 1 .. n + 3.
template <int TY, bool XB, bool YB>
__device__ __forceinline__ void step3_tile(const Problem& p, long long n, int par, int seg,
                                           int xa, int grp, int kb, int ke, int mask0,
                                           int mask1, int mask2) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nz = p.nz, nx = p.nx, ny = p.ny;
    const int j0 = (grp * WAVES + w) * TY;
    if (j0 >= ny) {                                            // uniform per wavefront
        for (int q = kb - 3; q <= ke + 2; ++q) __syncthreads(); // the others' barriers
        return;
    }
    const int lane = threadIdx.x & 63;
    const int own_lo = own_lo3(seg, xa), own_hi = own_hi3(seg, xa, nx);
    const int x0 = own_lo - 3;                                 // x of lane 0
    const int x = x0 + lane;
    const bool own = x >= own_lo && x < own_hi;
    const bool inb = !XB || (x >= 0 && x < nx);                // a grid cell
    const bool hold_x = XB && x == 0;                          // E_y, E_z on the x = 0 wall
    // A lane outside the grid reads the nearest cell of its row instead (so
    // every load of a row is unconditional).
    const int xc = XB ? min(max(x, 0), nx - 1) : x;
    auto row_ok = [&](int r) { return !YB || (j0 + r >= 0 && j0 + r < ny); };
    auto hold_y = [&](int r) { return YB && j0 + r == 0; };

    const size_t plane = (size_t)ny * p.pitch;
    const gptr<const float> fo = G((const float*)p.fbase[par]);
    const gptr<float> fw = G(p.fbase[par ^ 1]);
    const size_t fs = (size_t)p.fstride;
    // element offset of (component c, plane kk, row r) at lane 0: uniform
    // (modular arithmetic: rows and lanes before the grid are never accessed)
    auto base = [&](int c, int kk, int r) {
        return (size_t)c * fs + (size_t)kk * plane + (size_t)(long long)(j0 + r) * p.pitch +
               (size_t)(long long)x0;
    };
    const unsigned lo4 = 4u * (unsigned)(xc - x0);
    // Every row load is unconditional, as for the lanes: a row outside the
    // grid reads the nearest row inside it (row_in). Its values feed only
    // rows outside the grid (E there is zeroed after every E stage) and E_x,
    // E_z held on the y = 0 wall, at every stage.
    auto row_in = [&](int r) { return YB ? min(max(j0 + r, 0), ny - 1) - j0 : r; };
    auto ld = [&](int c, int kk, int r) {
        return *(gptr<const float>)(uniform3(fo + base(c, kk, row_in(r))) + lo4);
    };
    auto st = [&](int c, int kk, int r, float v) {
        *(gptr<float>)(uniform3(fw + base(c, kk, r)) + lo4) = v;
    };

    // ---- CPML: per-lane x coefficients, per-row y coefficients ----------
    const int npml = p.npml;
    const int xsl = XB && inb ? slab_index(x, nx, npml) : -1;
    Coef3 ex_c{0.f, 0.f, 1.f}, hx_c{0.f, 0.f, 1.f};
    if (xsl >= 0) {
        ex_c = Coef3{cx_tab(p, T_EB)[x], cx_tab(p, T_EC)[x], cx_tab(p, T_EK)[x]};
        hx_c = Coef3{cx_tab(p, T_HB)[x], cx_tab(p, T_HC)[x], cx_tab(p, T_HK)[x]};
    }
    // y slab index of the formed rows -2 .. TY+2 (uniform per row)
    constexpr int NR = YB ? TY + 6 : 1;
    int ysl_r[NR];
    if constexpr (YB) {
        ysl_r[0] = -1;
#pragma unroll
        for (int r = -2; r <= TY + 2; ++r)
            ysl_r[O + r] = row_ok(r) ? slab_index(j0 + r, ny, npml) : -1;
    }
    auto ysl = [&](int r) {
        if constexpr (YB) return ysl_r[O + r];
        return -1;
    };
    // The y coefficients of those rows (b, c, 1/κ at E and at H positions:
    // six per row) are copied into LDS once per tile and read where a stage
    // uses them, rather than held in scalar registers for the whole tile
    // (those tiles run short of them). Each wavefront reads only the rows it
    // wrote.
    extern __shared__ float2 amp_lds3[];
    constexpr int NCF = YB ? WAVES * (TY + 5) * 6 : 0;   // floats of coefficients
    float* const ycf = reinterpret_cast<float*>(amp_lds3);
    auto ycf_at = [&](int r, int t) { return (w * (TY + 5) + r + 2) * 6 + t; };
    if constexpr (YB) {
        if (lane < (TY + 5) * 6) {
            const int r = lane / 6 - 2, t = lane % 6;
            const int tab = t < 3 ? T_EB + t : T_HB + (t - 3);
            ycf[ycf_at(r, t)] = npml > 0 ? cy_tab(p, tab)[j0 + row_in(r)] : 0.f;
        }
    }
    // Without CPML (npml = 0) there are no memories: the memory loads below
    // then read the fields instead (in bounds), and nothing uses the values.
    const gptr<const float> po = npml > 0 ? G((const float*)p.pbase[par]) : fo;
    const gptr<float> pw = G(p.pbase[par ^ 1]);
    auto xq = [&](int kk, int r) { return ((size_t)kk * ny + (j0 + r)) * (2 * npml) + xsl; };
    auto yq = [&](int kk, int r) {
        return ((size_t)kk * (2 * npml) + ysl(r)) * p.pitch + xc;
    };
    auto ldx = [&](int q, int kk, int r) {   // x-slab memory q (used on slab lanes only)
        // unconditional: a lane off the slabs reads slab column 0 of the row
        // (the nearest row inside the grid), and the stages use no memory
        // off the slabs
        const size_t i = ((size_t)kk * ny + (j0 + row_in(r))) * (2 * npml) + max(xsl, 0);
        return po[psi_offset(p, q) + i];
    };
    auto stx = [&](int q, int kk, int r, float v) { pw[psi_offset(p, q) + xq(kk, r)] = v; };
    auto ldy = [&](int q, int kk, int r) {   // y-slab memory q (used on slab rows only)
        // unconditional, like the field rows: a row off the slabs reads slab
        // row 0 of its plane, and the stages use no memory off the slabs
        return po[psi_offset(p, q) + ((size_t)kk * (2 * npml) + max(ysl(r), 0)) * p.pitch + xc];
    };
    auto sty = [&](int q, int kk, int r, float v) { pw[psi_offset(p, q) + yq(kk, r)] = v; };

    // ---- antenna ------------------------------------------------------------
    const bool src = p.colmap != nullptr;
    int slot[TY + 6];
    slot[0] = -1;
#pragma unroll
    for (int r = -2; r <= TY + 2; ++r) {
        int v = -1;
        if (src && row_ok(r)) v = G(p.colmap)[(size_t)(j0 + r) * nx + xc];
        slot[O + r] = inb ? v : -1;
    }
    const gptr<const float2> amp = G(p.amp);
    // The antenna amplitudes of the rows a wavefront forms (-2 .. TY+2), one
    // float2 per (row, component, lane), staged in LDS once per tile and
    // read from there by every stage. The workgroup's rows are laid out
    // from row -2 of its first wavefront; rows two stacked wavefronts share
    // are written by both with the same values, and a wavefront reads only
    // rows it wrote itself.
    auto lds_at = [&](int r, int c) { return NCF / 2 + ((w * TY + r + 2) * 6 + c) * 64 + lane; };
    if (src) {
#pragma unroll
        for (int r = -2; r <= TY + 2; ++r) {
            if (slot[O + r] >= 0) {
                const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) amp_lds3[lds_at(r, c)] = ld2(a, c);
            }
        }
    }
    float2 tE[3], tH[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        tE[i] = src ? ldc2(p.tE, n + i) : make_float2(0.f, 0.f);
        tH[i] = src ? ldc2(p.tH, n + i) : make_float2(0.f, 0.f);
    }
    // e^{iβz} at the integer / half planes of a plane (z0, z1) times a time
    // factor
    auto phase = [&](float2 z0, float2 z1, float2 tt, float2& a0, float2& a1) {
        a0 = make_float2(0.f, 0.f);
        a1 = a0;
        if (src) {
            a0 = cmul(z0, tt);
            a1 = cmul(z1, tt);
        }
    };
    const gptr<double> fl = G(p.fl);
    auto accumulate = [&](int mask, int r, float vx, float vy, float vz) {
        const size_t pl = (size_t)(j0 + r) * nx + x, ps = (size_t)nx * ny;
        if (mask & FDTD_DIAG_EX2) fl[pl] = sq_acc(fl[pl], vx);
        if (mask & FDTD_DIAG_EY2) fl[ps + pl] = sq_acc(fl[ps + pl], vy);
        if (mask & FDTD_DIAG_EZ2) fl[2 * ps + pl] = sq_acc(fl[2 * ps + pl], vz);
    };
    // stored rows: inside the grid (uniform)
    auto row_st = [&](int r) { return j0 + r < ny; };

    // ---- the E and H cell updates (yee_cell.hpp's expressions) ----------
    // E at one row from the H differences; ψ_* hold the memories of the
    // old step and receive the new ones.
    auto e_upd = [&](int r, float& vx, float& vy, float& vz, float d_yhz, float d_zhy,
                     float d_zhx, float d_xhz, float d_xhy, float d_yhx, float& pyx, float& pzx,
                     float& pxy, float& pzy, bool do_y) {
        const bool hy0 = hold_y(r);
        float tx_hz = d_xhz, tx_hy = d_xhy, ty_hz = d_yhz, ty_hx = d_yhx;
        if constexpr (XB) {
            const float a = cpml_mem(ex_c.b, pyx, ex_c.c, d_xhz);
            const float b2 = cpml_mem(ex_c.b, pzx, ex_c.c, d_xhy);
            if (do_y && !hold_x) pyx = a;
            if (!hold_x && !hy0) pzx = b2;
            tx_hz = stretched(ex_c.k, d_xhz, pyx);
            tx_hy = stretched(ex_c.k, d_xhy, pzx);
        }
        if constexpr (YB) {
            if (ysl(r) >= 0) {
                const Coef3 cy{ycf[ycf_at(r, 0)], ycf[ycf_at(r, 1)], ycf[ycf_at(r, 2)]};
                if (!hy0) pxy = cpml_mem(cy.b, pxy, cy.c, d_yhz);
                const float b2 = cpml_mem(cy.b, pzy, cy.c, d_yhx);
                if (!hy0 && !hold_x) pzy = b2;
                ty_hz = stretched(cy.k, d_yhz, pxy);
                ty_hx = stretched(cy.k, d_yhx, pzy);
            }
        }
        if (!hy0) vx += curl_pair(p.sy, ty_hz, p.sz, d_zhy);
        if (do_y && !hold_x) vy += curl_pair(p.sz, d_zhx, p.sx, tx_hz);
        if (!hold_x && !hy0) vz += curl_pair(p.sx, tx_hy, p.sy, ty_hx);
    };
    auto h_upd = [&](int r, float& vx, float& vy, float& vz, float d_yez, float d_zey,
                     float d_zex, float d_xez, float d_xey, float d_yex, float& pyx, float& pzx,
                     float& pxy, float& pzy, bool do_y) {
        float tx_ez = d_xez, tx_ey = d_xey, ty_ez = d_yez, ty_ex = d_yex;
        if constexpr (XB) {
            if (do_y) pyx = cpml_mem(hx_c.b, pyx, hx_c.c, d_xez);
            pzx = cpml_mem(hx_c.b, pzx, hx_c.c, d_xey);
            tx_ez = stretched(hx_c.k, d_xez, pyx);
            tx_ey = stretched(hx_c.k, d_xey, pzx);
        }
        if constexpr (YB) {
            if (ysl(r) >= 0) {
                const Coef3 cy{ycf[ycf_at(r, 3)], ycf[ycf_at(r, 4)], ycf[ycf_at(r, 5)]};
                pxy = cpml_mem(cy.b, pxy, cy.c, d_yez);
                pzy = cpml_mem(cy.b, pzy, cy.c, d_yex);
                ty_ez = stretched(cy.k, d_yez, pxy);
                ty_ex = stretched(cy.k, d_yex, pzy);
            }
        }
        vx -= curl_pair(p.sy, ty_ez, p.sz, d_zey);
        if (do_y) vy -= curl_pair(p.sz, d_zex, p.sx, tx_ez);
        vz -= curl_pair(p.sx, tx_ey, p.sy, ty_ex);
    };
    // E beyond the last cell of the grid is zero (the PEC wall)
    auto zero_out = [&](int r, float& vx, float& vy, float& vz) {
        if ((XB && !inb) || (YB && !row_ok(r))) vx = vy = vz = 0.f;
    };
    // One E stage in place on rows [ra, rb] (E_y on [ra, rb - 1]): E from H
    // (plane k), Hp (plane k - 1) and the CPML memories of those rows, plus
    // the source.
    auto e_stage = [&](float* vx, float* vy, float* vz, const float* hx, const float* hy,
                       const float* hz, const float* px, const float* py, float* myx,
                       float* mzx, float* mxy, float* mzy, int ra, int rb, float2 pt0,
                       float2 pt1) {
#pragma unroll
        for (int r = -2; r <= TY + 2; ++r) {
            if (r < ra || r > rb) continue;
            const int i = O + r;
            const float hz_im = lane_below(hz[i]);
            const float hy_im = lane_below(hy[i]);
            float dm = 0.f;
            const bool do_y = r < rb;
            e_upd(r, vx[i], vy[i], vz[i], hz[i] - hz[i - 1], hy[i] - py[i], hx[i] - px[i],
                  hz[i] - hz_im, hy[i] - hy_im, hx[i] - hx[i - 1], XB ? myx[i] : dm,
                  XB ? mzx[i] : dm, YB ? mxy[i] : dm, YB ? mzy[i] : dm, do_y);
            if (slot[i] >= 0) {
                vx[i] += cmul_re(amp_lds3[lds_at(r, EX)], pt0);
                vz[i] += cmul_re(amp_lds3[lds_at(r, EZ)], pt1);
                if (do_y) vy[i] += cmul_re(amp_lds3[lds_at(r, EY)], pt0);
            }
            zero_out(r, vx[i], vy[i], vz[i]);
        }
    };
    // One H stage in place on rows [ra, rb] (H_y on [ray, rb]): H from E
    // (plane k), Eu (plane k + 1) and the CPML memories of those rows, plus
    // the source.
    auto h_stage = [&](float* vx, float* vy, float* vz, const float* ex, const float* ey,
                       const float* ez, const float* ux, const float* uy, float* myx,
                       float* mzx, float* mxy, float* mzy, int ra, int rb, int ray, float2 qt0,
                       float2 qt1) {
#pragma unroll
        for (int r = -2; r <= TY + 2; ++r) {
            if (r < ra || r > rb) continue;
            const int i = O + r;
            const float ey_ip = lane_above(ey[i]);
            const float ez_ip = lane_above(ez[i]);
            float dm = 0.f;
            const bool do_y = r >= ray;
            h_upd(r, vx[i], vy[i], vz[i], ez[i + 1] - ez[i], uy[i] - ey[i], ux[i] - ex[i],
                  ez_ip - ez[i], ey_ip - ey[i], ex[i + 1] - ex[i], XB ? myx[i] : dm,
                  XB ? mzx[i] : dm, YB ? mxy[i] : dm, YB ? mzy[i] : dm, do_y);
            if (slot[i] >= 0) {
                vx[i] += cmul_re(amp_lds3[lds_at(r, HX)], qt1);
                if (do_y) vy[i] += cmul_re(amp_lds3[lds_at(r, HY)], qt1);
                vz[i] += cmul_re(amp_lds3[lds_at(r, HZ)], qt0);
            }
        }
    };

    constexpr int R = TY + 6;
    // carried planes: H^{n+1/2}(q-1), E^{n+1}(q-1), H^{n+3/2}(q-2),
    // E^{n+2}(q-2), H^{n+5/2}(q-3), E^{n+3}(q-3)
    float hpx[R], hpy[R], hpz[R], e1x[R], e1y[R], e1z[R];
    float h1x[R], h1y[R], h1z[R], e2x[R], e2y[R], e2z[R];
    float h2x[R], h2y[R], h2z[R], e3x[R], e3y[R], e3z[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        hpx[i] = hpy[i] = hpz[i] = e1x[i] = e1y[i] = e1z[i] = 0.f;
        h1x[i] = h1y[i] = h1z[i] = e2x[i] = e2y[i] = e2z[i] = 0.f;
        h2x[i] = h2y[i] = h2z[i] = e3x[i] = e3y[i] = e3z[i] = 0.f;
    }
    // carried CPML memories: ψ_E^{n+1}(q-1), ψ_E^{n+2}(q-2) and
    // ψ_H^{n+3/2}(q-2), ψ_H^{n+5/2}(q-3)
    constexpr int PX = XB ? R : 1, PY = YB ? R : 1;
    float qe_yx[PX], qe_zx[PX], re_yx[PX], re_zx[PX];
    float qh_yx[PX], qh_zx[PX], rh_yx[PX], rh_zx[PX];
    float qe_xy[PY], qe_zy[PY], re_xy[PY], re_zy[PY];
    float qh_xy[PY], qh_zy[PY], rh_xy[PY], rh_zy[PY];
#pragma unroll
    for (int i = 0; i < PX; ++i)
        qe_yx[i] = qe_zx[i] = re_yx[i] = re_zx[i] = qh_yx[i] = qh_zx[i] = rh_yx[i] = rh_zx[i] = 0.f;
#pragma unroll
    for (int i = 0; i < PY; ++i)
        qe_xy[i] = qe_zy[i] = re_xy[i] = re_zy[i] = qh_xy[i] = qh_zy[i] = rh_xy[i] = rh_zy[i] = 0.f;

    int kq = kb - 3;
    while (kq < 0) kq += nz;
    kq %= nz;
    int kq1 = 0, kq2 = 0, kq3 = 0;   // planes of q-1, q-2, q-3
    // e^{iβz} of planes q-1, q-2 and q-3 (integer, half plane), carried
    float2 za0 = make_float2(0.f, 0.f), za1 = za0, zb0 = za0, zb1 = za0, zc0 = za0, zc1 = za0;
    for (int q = kb - 3; q <= ke + 2; ++q) {
        // The four wavefronts of the workgroup start each plane together, so
        // the halo rows one loads are the rows its neighbour loads in the
        // same window (every wavefront passes this barrier equally often).
        __syncthreads();
        // ---- plane q of E^n and H^{n+1/2} --------------------------------
        float hx[R], hy[R], hz[R], ex[R], ey[R], ez[R];
#pragma unroll
        for (int r = -3; r <= TY + 2; ++r) {
            hx[O + r] = ld(HX, kq, r);
            hz[O + r] = ld(HZ, kq, r);
            hy[O + r] = r >= -2 ? ld(HY, kq, r) : 0.f;
            ex[O + r] = r >= -2 ? ld(EX, kq, r) : 0.f;
            ez[O + r] = r >= -2 ? ld(EZ, kq, r) : 0.f;
            ey[O + r] = r >= -2 && r <= TY + 1 ? ld(EY, kq, r) : 0.f;
        }
        float2 zq0 = make_float2(0.f, 0.f), zq1 = zq0;   // e^{iβz} of plane q
        if (src) {
            zq0 = ldc2(p.zph, 2 * kq);
            zq1 = ldc2(p.zph, 2 * kq + 1);
        }
        // CPML memories of the first stage, issued with the field loads:
        // ψ_E^n(q) and ψ_H^{n+1/2}(q-1)
        float pe_yx[PX], pe_zx[PX], pe_xy[PY], pe_zy[PY];
        float ph_yx[PX], ph_zx[PX], ph_xy[PY], ph_zy[PY];
#pragma unroll
        for (int r = -3; r <= TY + 2; ++r) {
            const bool fe = r >= -2, fh = r >= -2 && r <= TY + 1;   // E1 / H1 rows
            if constexpr (XB) {
                pe_yx[O + r] = fe ? ldx(P_EYX, kq, r) : 0.f;
                pe_zx[O + r] = fe ? ldx(P_EZX, kq, r) : 0.f;
                ph_yx[O + r] = fh ? ldx(P_HYX, kq1, r) : 0.f;
                ph_zx[O + r] = fh ? ldx(P_HZX, kq1, r) : 0.f;
            }
            if constexpr (YB) {
                pe_xy[O + r] = fe ? ldy(P_EXY, kq, r) : 0.f;
                pe_zy[O + r] = fe ? ldy(P_EZY, kq, r) : 0.f;
                ph_xy[O + r] = fh ? ldy(P_HXY, kq1, r) : 0.f;
                ph_zy[O + r] = fh ? ldy(P_HZY, kq1, r) : 0.f;
            }
        }
        float2 pt0, pt1;

        // ---- E^{n+1}(q), rows -2 .. TY+2, in place -----------------------
        phase(zq0, zq1, tE[0], pt0, pt1);
        e_stage(ex, ey, ez, hx, hy, hz, hpx, hpy, pe_yx, pe_zx, pe_xy, pe_zy, -2, TY + 2, pt0,
                pt1);
        if (mask0 && kq == p.plane && q >= kb && q < ke && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                if (row_st(r)) accumulate(mask0, r, ex[O + r], ey[O + r], ez[O + r]);
        }

        // ---- H^{n+3/2}(q-1), rows -2 .. TY+1 -------------------------------
        float gx[R], gy[R], gz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            gx[i] = hpx[i];
            gy[i] = hpy[i];
            gz[i] = hpz[i];
        }
        phase(za0, za1, tH[0], pt0, pt1);
        h_stage(gx, gy, gz, e1x, e1y, e1z, ex, ey, ph_yx, ph_zx, ph_xy, ph_zy, -2, TY + 1, -1,
                pt0, pt1);

        // ---- E^{n+2}(q-1), rows -1 .. TY+1 ---------------------------------
        float fx[R], fy[R], fz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            fx[i] = e1x[i];
            fy[i] = e1y[i];
            fz[i] = e1z[i];
        }
        phase(za0, za1, tE[1], pt0, pt1);
        e_stage(fx, fy, fz, gx, gy, gz, h1x, h1y, qe_yx, qe_zx, qe_xy, qe_zy, -1, TY + 1, pt0,
                pt1);
        if (mask1 && kq1 == p.plane && q - 1 >= kb && q - 1 < ke && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                if (row_st(r)) accumulate(mask1, r, fx[O + r], fy[O + r], fz[O + r]);
        }

        // ---- H^{n+5/2}(q-2), rows -1 .. TY ---------------------------------
        float ux[R], uy[R], uz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            ux[i] = h1x[i];
            uy[i] = h1y[i];
            uz[i] = h1z[i];
        }
        phase(zb0, zb1, tH[1], pt0, pt1);
        h_stage(ux, uy, uz, e2x, e2y, e2z, fx, fy, qh_yx, qh_zx, qh_xy, qh_zy, -1, TY, 0, pt0,
                pt1);

        // ---- E^{n+3}(q-2), rows 0 .. TY --------------------------------------
        float vx[R], vy[R], vz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            vx[i] = e2x[i];
            vy[i] = e2y[i];
            vz[i] = e2z[i];
        }
        phase(zb0, zb1, tE[2], pt0, pt1);
        e_stage(vx, vy, vz, ux, uy, uz, h2x, h2y, re_yx, re_zx, re_xy, re_zy, 0, TY, pt0, pt1);
        if (q - 2 >= kb && q - 2 < ke && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (!row_st(r)) continue;
                st(EX, kq2, r, vx[O + r]);
                st(EY, kq2, r, vy[O + r]);
                st(EZ, kq2, r, vz[O + r]);
                if constexpr (XB) {
                    if (xsl >= 0) {
                        stx(P_EYX, kq2, r, re_yx[O + r]);
                        stx(P_EZX, kq2, r, re_zx[O + r]);
                    }
                }
                if constexpr (YB) {
                    if (ysl(r) >= 0) {
                        sty(P_EXY, kq2, r, re_xy[O + r]);
                        sty(P_EZY, kq2, r, re_zy[O + r]);
                    }
                }
            }
            if (mask2 && kq2 == p.plane) {
#pragma unroll
                for (int r = 0; r < TY; ++r)
                    if (row_st(r)) accumulate(mask2, r, vx[O + r], vy[O + r], vz[O + r]);
            }
        }

        // ---- H^{n+7/2}(q-3), rows 0 .. TY-1 ---------------------------------
        if (q - 3 >= kb && q - 3 < ke) {
            float wx[R], wy[R], wz[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                wx[i] = h2x[i];
                wy[i] = h2y[i];
                wz[i] = h2z[i];
            }
            phase(zc0, zc1, tH[2], pt0, pt1);
            h_stage(wx, wy, wz, e3x, e3y, e3z, vx, vy, rh_yx, rh_zx, rh_xy, rh_zy, 0, TY - 1, 0,
                    pt0, pt1);
            if (own) {
#pragma unroll
                for (int r = 0; r < TY; ++r) {
                    if (!row_st(r)) continue;
                    st(HX, kq3, r, wx[O + r]);
                    st(HY, kq3, r, wy[O + r]);
                    st(HZ, kq3, r, wz[O + r]);
                    if constexpr (XB) {
                        if (xsl >= 0) {
                            stx(P_HYX, kq3, r, rh_yx[O + r]);
                            stx(P_HZX, kq3, r, rh_zx[O + r]);
                        }
                    }
                    if constexpr (YB) {
                        if (ysl(r) >= 0) {
                            sty(P_HXY, kq3, r, rh_xy[O + r]);
                            sty(P_HZY, kq3, r, rh_zy[O + r]);
                        }
                    }
                }
            }
        }

        // ---- rotate ----------------------------------------------------------
#pragma unroll
        for (int i = 0; i < R; ++i) {
            hpx[i] = hx[i];
            hpy[i] = hy[i];
            hpz[i] = hz[i];
            e1x[i] = ex[i];
            e1y[i] = ey[i];
            e1z[i] = ez[i];
            h1x[i] = gx[i];
            h1y[i] = gy[i];
            h1z[i] = gz[i];
            e2x[i] = fx[i];
            e2y[i] = fy[i];
            e2z[i] = fz[i];
            h2x[i] = ux[i];
            h2y[i] = uy[i];
            h2z[i] = uz[i];
            e3x[i] = vx[i];
            e3y[i] = vy[i];
            e3z[i] = vz[i];
        }
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            if constexpr (XB) {
                re_yx[i] = qe_yx[i];
                re_zx[i] = qe_zx[i];
                qe_yx[i] = pe_yx[i];
                qe_zx[i] = pe_zx[i];
                rh_yx[i] = qh_yx[i];
                rh_zx[i] = qh_zx[i];
                qh_yx[i] = ph_yx[i];
                qh_zx[i] = ph_zx[i];
            }
        }
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            if constexpr (YB) {
                re_xy[i] = qe_xy[i];
                re_zy[i] = qe_zy[i];
                qe_xy[i] = pe_xy[i];
                qe_zy[i] = pe_zy[i];
                rh_xy[i] = qh_xy[i];
                rh_zy[i] = qh_zy[i];
                qh_xy[i] = ph_xy[i];
                qh_zy[i] = ph_zy[i];
            }
        }
        zc0 = zb0;
        zc1 = zb1;
        zb0 = za0;
        zb1 = za1;
        za0 = zq0;
        za1 = zq1;
        kq3 = kq2;
        kq2 = kq1;
        kq1 = kq;
        kq = kq + 1 == nz ? 0 : kq + 1;
    }
}

// Block b runs on XCD b % 8; blocks are remapped so that each XCD takes a
// contiguous run of tiles (consecutive segments of a row group and z chunk
// share halo rows in that XCD's L2).
// Waves per SIMD asked of the register allocator: corner tiles carry both
// walls' CPML state through three stages and at two waves per SIMD spill to
// scratch memory; at one they keep it in registers (VGPRs and AGPRs).
template <int TY, bool XB, bool YB>
constexpr int step3_waves() {
    return (XB && YB) ? 1 : 2;
}

template <int TY, bool XB, bool YB>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(step3_waves<TY, XB, YB>())))
step3_kernel(Problem p, long long n, int par, Launch3 L, int nblocks_padded, int mask0,
             int mask1, int mask2) {
    const int nsl = count3(L.seg), ngl = count3(L.grp);
    const int ntile = nsl * ngl;
    const int lb = (blockIdx.x % 8) * (nblocks_padded / 8) + blockIdx.x / 8;
    if (lb >= ntile * L.ncz) return;
    const int t = lb % ntile;
    const int kb = (lb / ntile) * L.cz;
    step3_tile<TY, XB, YB>(p, n, par, at3(L.seg, t % nsl), L.xa, at3(L.grp, t / nsl), kb,
                           min(kb + L.cz, p.nz), mask0, mask1, mask2);
}

// LDS of the staged antenna amplitudes of one workgroup: the 4 TY + 5 rows
// its wavefronts form, six components, 64 lanes (39 KiB at TY = 2, 63 KiB at
// TY = 4).
constexpr unsigned amp_lds_bytes3(int ty) {
    return (unsigned)((WAVES * ty + 5) * 6 * 64 * sizeof(float2));
}
// LDS of the y CPML coefficients of a y-boundary or corner workgroup: six
// per formed row of each wavefront (672 B at TY = 2), ahead of the
// amplitudes.
constexpr unsigned ycf_lds_bytes3(int ty) {
    return (unsigned)(WAVES * (ty + 5) * 6 * sizeof(float));
}

// Segments and row groups whose tiles form only regular cells (an interval
// each, possibly empty).
struct Plan3 {
    int nseg, ngrp, s_lo, s_hi, g_lo, g_hi, cz, ncz, xa;
};

Plan3 plan3(const Problem& p, int rows, int zchunk) {
    Plan3 P{};
    const int G = WAVES * rows;
    // The cells left over from whole 58-cell segments are split between the
    // two end segments (which hold the walls and CPML slabs), so that no
    // third, nearly empty segment runs the boundary code: with nx = 58 q + r
    // (0 < r < 58) the first segment owns (58 + r) / 2 cells, the last the
    // rest of 58 + r.
    const int r = p.nx % OWN;
    P.xa = p.nx <= OWN ? p.nx : r == 0 ? OWN : (OWN + r) / 2;
    P.nseg = 1 + (p.nx - P.xa + OWN - 1) / OWN;
    P.ngrp = (p.ny + G - 1) / G;
    const int m = std::max(p.npml, 1);
    // segment s: lanes x = own_lo3(s) - 3 + l; lanes 1..63 must be regular
    // cells, lane 0 inside the grid
    P.s_lo = P.nseg;
    P.s_hi = P.nseg;
    for (int s = 0; s < P.nseg; ++s) {
        const int x0 = own_lo3(s, P.xa) - 3;
        const bool reg = x0 >= 0 && x0 + 1 >= m && x0 + 63 <= p.nx - p.npml - 1;
        if (reg && P.s_lo == P.nseg) P.s_lo = s;
        if (reg) P.s_hi = s + 1;
    }
    if (P.s_lo >= P.s_hi) P.s_lo = P.s_hi = P.nseg;
    // row group g: formed rows g G - 2 .. g G + G + 2 regular (row g G - 3 is
    // only read)
    P.g_lo = P.ngrp;
    P.g_hi = P.ngrp;
    for (int g = 0; g < P.ngrp; ++g) {
        const bool reg = g * G - 2 >= m && g * G + G + 2 <= p.ny - p.npml - 1;
        if (reg && P.g_lo == P.ngrp) P.g_lo = g;
        if (reg) P.g_hi = g + 1;
    }
    if (P.g_lo >= P.g_hi) P.g_lo = P.g_hi = P.ngrp;
    P.cz = zchunk > 0 ? std::min(zchunk, p.nz) : p.nz;
    P.ncz = (p.nz + P.cz - 1) / P.cz;
    return P;
}

template <int TY, bool XB, bool YB>
hipError_t launch_class3(const Problem& p, long long n, int parity, const Launch3& L, int mask0,
                         int mask1, int mask2, hipStream_t s, LaunchTimer* timer,
                         const char* name) {
    const int nt = count3(L.seg) * count3(L.grp) * L.ncz;
    if (nt <= 0) return hipSuccess;
    const int nbp = (nt + 7) / 8 * 8;
    if (timer) timer->mark_on(name, s);
    const unsigned lds = (p.colmap ? amp_lds_bytes3(TY) : 0u) + (YB ? ycf_lds_bytes3(TY) : 0u);
    hipLaunchKernelGGL((step3_kernel<TY, XB, YB>), dim3(nbp), dim3(64 * WAVES), lds, s, p, n,
                       parity, L, nbp, mask0, mask1, mask2);
    hipError_t e = hipGetLastError();
    if (timer) timer->mark_on(nullptr, s);
    return e;
}

// The four classes touch disjoint cells: with side streams the boundary
// classes run beside the interior launch, forked from and joined back into
// s by events.
template <int TY>
hipError_t launch_rows3(const Problem& p, long long n, int parity, int zchunk, int mask0,
                        int mask1, int mask2, hipStream_t s, LaunchTimer* timer,
                        const SideStreams* side) {
    const Plan3 P = plan3(p, TY, zchunk);
    const Span3 s_int{P.s_lo, P.s_hi, 0, 0}, s_bnd{0, P.s_lo, P.s_hi, P.nseg};
    const Span3 g_int{P.g_lo, P.g_hi, 0, 0}, g_bnd{0, P.g_lo, P.g_hi, P.ngrp};
    const bool fork = side != nullptr;
    hipStream_t sx = s, sy = s, sc = s;
    hipError_t e;
    if (fork) {
        e = hipEventRecord(side->fork, s);
        for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipStreamWaitEvent(side->s[q], side->fork, 0);
        if (e != hipSuccess) return e;
        sx = side->s[0];
        sy = side->s[1];
        sc = side->s[2];
    }
    // The corner and y-boundary classes hold few tiles: shorter z chunks
    // give them more workgroups at the cost of re-reading five planes per
    // chunk.
    const int czc = std::min(P.cz, 16), czy = std::min(P.cz, 32);
    e = launch_class3<TY, true, true>(p, n, parity,
                                      Launch3{s_bnd, g_bnd, czc, (p.nz + czc - 1) / czc, P.xa},
                                      mask0, mask1, mask2, sc, timer, "step3_corner");
    if (e == hipSuccess)
        e = launch_class3<TY, false, true>(
            p, n, parity, Launch3{s_int, g_bnd, czy, (p.nz + czy - 1) / czy, P.xa}, mask0, mask1,
            mask2, sy, timer, "step3_ybnd");
    if (e == hipSuccess)
        e = launch_class3<TY, true, false>(p, n, parity,
                                           Launch3{s_bnd, g_int, P.cz, P.ncz, P.xa}, mask0,
                                           mask1, mask2, sx, timer, "step3_xbnd");
    if (e == hipSuccess)
        e = launch_class3<TY, false, false>(p, n, parity,
                                            Launch3{s_int, g_int, P.cz, P.ncz, P.xa}, mask0,
                                            mask1, mask2, s, timer, "step3_interior");
    if (fork) {
        for (int q = 0; q < 3; ++q) {
            hipError_t f = hipEventRecord(side->join[q], side->s[q]);
            if (f == hipSuccess) f = hipStreamWaitEvent(s, side->join[q], 0);
            if (e == hipSuccess) e = f;
        }
    }
    return e;
}

}  // namespace

long long step3_interior_cells(const Problem& p, int rows) {
    const Plan3 P = plan3(p, rows, 0);
    if (P.s_lo >= P.s_hi || P.g_lo >= P.g_hi) return 0;
    const long long xs = own_hi3(P.s_hi - 1, P.xa, p.nx) - own_lo3(P.s_lo, P.xa);
    const long long ys = std::min(WAVES * rows * P.g_hi, p.ny) - WAVES * rows * P.g_lo;
    return xs * ys * p.nz;
}

hipError_t launch_step3(const Problem& p, long long n, int parity, int rows, int zchunk,
                        int mask0, int mask1, int mask2, hipStream_t s, LaunchTimer* timer,
                        const SideStreams* side) {
    if (p.periodic) return hipErrorInvalidValue;
    if (rows == 2)
        return launch_rows3<2>(p, n, parity, zchunk, mask0, mask1, mask2, s, timer, side);
    if (rows == 4)
        return launch_rows3<4>(p, n, parity, zchunk, mask0, mask1, mask2, s, timer, side);
    return hipErrorInvalidValue;
}

}  // namespace bfdtd
