// Two-step Yee kernel over the whole grid (temporal blocking): one pass over
// the fields advances every cell by two leapfrog steps, E^n, H^{n+1/2} ->
// E^{n+2}, H^{n+5/2}, CPML memories ψ^n -> ψ^{n+2}, with the antenna's soft
// source (§4) folded in: the old ping-pong buffers are read once and the new
// ones written once, 48 B of field traffic per cell for two cell-updates.
// Each cell is formed with the expressions of the one-step cell code
// (yee_cell.hpp), in the same order, so a pair equals two one-step launches
// bit for bit.
//
// Work decomposition (CDNA4, wave64). A wavefront reads a block of 64 x
// cells (lane l at x = 60 s - 2 + l for x segment s) by TY + 4 rows
// (j0 - 2 .. j0 + TY + 1) and marches along z. The intermediate step is
// formed in registers on every lane and row it can be formed on, so the
// second step needs nothing from other wavefronts:
//   x: neighbours move between lanes with DPP wavefront shifts; lanes 0-1
//      and 62-63 are halo and the wavefront stores lanes 2..61 (60 cells).
//   y: E^{n+1} is formed on rows -1 .. TY+1, H^{n+3/2} on rows -1 .. TY,
//      E^{n+2} on rows 0 .. TY, H^{n+5/2} on the TY stored rows.
//   z: at plane q the pipeline forms E^{n+1}(q), H^{n+3/2}(q-1),
//      E^{n+2}(q-1) and H^{n+5/2}(q-2), keeping one plane of each in
//      registers; a chunk [kb, ke) reads planes kb-2 .. ke+1 (z is periodic).
// Waits. On this chip one counter tracks a wavefront's vector-memory loads
// and stores together, so waiting for any vector load also waits for every
// older load and store. A plane therefore issues all its vector loads at
// its start (fields and CPML memories; interior tiles load the next plane's
// H rows at the end of the previous one, beside its stores), reads the z
// phases e^{iβz} with scalar loads and the antenna amplitudes from LDS, and
// waits on vector memory only for the plane's own field loads.
// A workgroup stacks four wavefronts in y that start every plane together
// (one barrier per plane): a row group of 4 TY rows.
//
// Tiles (segment, row group) fall in four classes, each its own launch and
// instantiation, so that the interior keeps the register budget of plain
// Yee updates:
//   interior: every formed cell is regular (no wall, no CPML);
//   XB: formed lanes reach a wall or an x CPML slab (per-lane CPML
//       coefficients, held E_y/E_z at x = 0, zero E beyond x = nx - 1);
//   YB: formed rows reach a wall or a y slab (per-row coefficients, held
//       E_x/E_z at y = 0, zero E beyond y = ny - 1);
//   XB and YB (the corners).
// On a boundary lane outside the slabs the CPML form runs with b = c = 0 and
// 1/κ = 1, which gives the plain update's value exactly.
//
// The x-slab memories are [z][y][2 npml], the y-slab memories
// [z][2 npml][pitch]; a pair reads those of parity par and writes those of
// parity par ^ 1, like the fields.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int WAVES = 4;   // wavefronts per workgroup, stacked in y
constexpr int OWN = 60;    // x cells stored per wavefront (lanes 2..61)
constexpr int O = 2;       // register index of row r is r + O (rows -2 .. TY+1)

// A wave-uniform global pointer as a byte pointer held in scalar registers.
template <typename T>
__device__ __forceinline__ gptr<char> uniform(gptr<T> q) {
    const unsigned long long a = (unsigned long long)q;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    return (gptr<char>)(((unsigned long long)hi << 32) | lo);
}

// Cross-lane moves by one lane (DPP wavefront shifts: a VALU operand
// modifier, no LDS round trip). Lanes without a source keep their own value.
__device__ __forceinline__ float from_lower(float v) {   // lane l gets lane l - 1
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_upper(float v) {   // lane l gets lane l + 1
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x130, 0xf, 0xf, false));
}

// Indices [a0, a1) then [b0, b1).
struct Span {
    int a0, a1, b0, b1;
};
__host__ __device__ __forceinline__ int span_count(const Span& s) {
    return (s.a1 - s.a0) + (s.b1 - s.b0);
}
__device__ __forceinline__ int span_at(const Span& s, int i) {
    const int na = s.a1 - s.a0;
    return i < na ? s.a0 + i : s.b0 + (i - na);
}

// One launch: its x segments and row groups, and the z chunks.
struct Launch2 {
    Span seg, grp;
    int cz, ncz;
};

// CPML coefficients of one position: b, c and 1/κ (identity outside a slab).
struct Coef {
    float b, c, k;
};

// Waves per SIMD asked of the register allocator (at least).
template <int TY, bool XB, bool YB>
constexpr int step2_waves() {
    return 2;
}

// One tile: x segment seg, row group grp, planes [kb, ke) of problem p,
// advanced from step n (parity par) to n + 2.
template <int TY, bool XB, bool YB>
__device__ __forceinline__ void step2_tile(const Problem& p, long long n, int par, int seg,
                                           int grp, int kb, int ke, int mask0, int mask1) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nz = p.nz, nx = p.nx, ny = p.ny;
    const int j0 = (grp * WAVES + w) * TY;
    if (j0 >= ny) {                                            // uniform per wavefront
        for (int q = kb - 2; q <= ke + 1; ++q) __syncthreads(); // the others' barriers
        return;
    }
    const int lane = threadIdx.x & 63;
    const int x0 = OWN * seg - 2;                              // x of lane 0
    const int x = x0 + lane;
    const int own_lo = OWN * seg, own_hi = min(own_lo + OWN, nx);
    const bool own = x >= own_lo && x < own_hi;
    const bool inb = !XB || (x >= 0 && x < nx);                // a grid cell
    const bool hold_x = XB && x == 0;                          // E_y, E_z on the x = 0 wall
    // A lane outside the grid reads the nearest cell of its row instead (so
    // every load of a row is unconditional): its values feed only cells
    // outside the grid or held on the wall, and E outside is zeroed after
    // every E update.
    const int xc = XB ? min(max(x, 0), nx - 1) : x;
    // rows: inside the grid, and on the y = 0 wall (uniform per row)
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
    // rows outside the grid (E there is zeroed after every E update) and
    // E_x, E_z held on the y = 0 wall. A load under a per-row branch can
    // make the compiler wait for it before the next one issues.
    auto row_in = [&](int r) { return YB ? min(max(j0 + r, 0), ny - 1) - j0 : r; };
    auto ld = [&](int c, int kk, int r) {
        return *(gptr<const float>)(uniform(fo + base(c, kk, row_in(r))) + lo4);
    };
    // plain stores: a tile stores 60 cells of a row, so lines at tile edges
    // are written by two tiles and merge in L2
    auto st = [&](int c, int kk, int r, float v) {
        *(gptr<float>)(uniform(fw + base(c, kk, r)) + lo4) = v;
    };

    // ---- CPML: per-lane x coefficients, per-row y coefficients ----------
    const int npml = p.npml;
    const int xsl = XB && inb ? slab_index(x, nx, npml) : -1;
    Coef ex_c{0.f, 0.f, 1.f}, hx_c{0.f, 0.f, 1.f};
    if (xsl >= 0) {
        ex_c = Coef{cx_tab(p, T_EB)[x], cx_tab(p, T_EC)[x], cx_tab(p, T_EK)[x]};
        hx_c = Coef{cx_tab(p, T_HB)[x], cx_tab(p, T_HC)[x], cx_tab(p, T_HK)[x]};
    }
    // y slab index and coefficients of rows -1 .. TY+1 (uniform per row)
    constexpr int NR = YB ? TY + 4 : 1;
    int ysl_r[NR];
    Coef eyc[NR], hyc[NR];
    if constexpr (YB) {
#pragma unroll
        for (int r = -1; r <= TY + 1; ++r) {
            const int j = j0 + r;
            ysl_r[O + r] = row_ok(r) ? slab_index(j, ny, npml) : -1;
            eyc[O + r] = Coef{0.f, 0.f, 1.f};
            hyc[O + r] = Coef{0.f, 0.f, 1.f};
            if (ysl_r[O + r] >= 0) {
                eyc[O + r] = Coef{cy_tab(p, T_EB)[j], cy_tab(p, T_EC)[j], cy_tab(p, T_EK)[j]};
                hyc[O + r] = Coef{cy_tab(p, T_HB)[j], cy_tab(p, T_HC)[j], cy_tab(p, T_HK)[j]};
            }
        }
    }
    auto ysl = [&](int r) {
        if constexpr (YB) return ysl_r[O + r];
        return -1;
    };
    // Without CPML (npml = 0) there are no memories: the memory loads below
    // then read the fields instead (in bounds), and nothing uses the values.
    const gptr<const float> po = npml > 0 ? G((const float*)p.pbase[par]) : fo;
    const gptr<float> pw = G(p.pbase[par ^ 1]);
    auto xq = [&](int kk, int r) { return ((size_t)kk * ny + (j0 + r)) * (2 * npml) + xsl; };
    auto yq = [&](int kk, int r) {
        return ((size_t)kk * (2 * npml) + ysl(r)) * p.pitch + xc;
    };
    // CPML memory loads are unconditional too: a lane or row off the slabs
    // reads slab column or row 0 (of the nearest row inside the grid), and
    // no update uses a memory off the slabs.
    auto ldx = [&](int q, int kk, int r) {   // x-slab memory q (used on slab lanes only)
        const size_t i = ((size_t)kk * ny + (j0 + row_in(r))) * (2 * npml) + max(xsl, 0);
        return po[psi_offset(p, q) + i];
    };
    auto stx = [&](int q, int kk, int r, float v) { pw[psi_offset(p, q) + xq(kk, r)] = v; };
    auto ldy = [&](int q, int kk, int r) {   // y-slab memory q (used on slab rows only)
        return po[psi_offset(p, q) + ((size_t)kk * (2 * npml) + max(ysl(r), 0)) * p.pitch + xc];
    };
    auto sty = [&](int q, int kk, int r, float v) { pw[psi_offset(p, q) + yq(kk, r)] = v; };

    // ---- antenna ------------------------------------------------------------
    const bool src = p.colmap != nullptr;
    int slot[TY + 4];
#pragma unroll
    for (int r = -1; r <= TY + 1; ++r)
    {
        int v = -1;
        if (src && row_ok(r)) v = G(p.colmap)[(size_t)(j0 + r) * nx + xc];
        slot[O + r] = inb ? v : -1;
    }
    const gptr<const float2> amp = G(p.amp);
    // The antenna amplitudes of the rows a wavefront forms (-1 .. TY+1), one
    // float2 per (row, component, lane), staged in LDS once per tile: the
    // stages read them with LDS loads, whose waits leave the vector-memory
    // counter alone (a vector load's wait would also wait for the field
    // loads and stores in flight). The workgroup's rows are laid out from
    // row -1 of its first wavefront; rows two stacked wavefronts share are
    // written by both with the same values, and a wavefront reads only rows
    // it wrote itself.
    extern __shared__ float2 amp_lds[];
    auto lds_at = [&](int r, int c) { return ((w * TY + r + 1) * 6 + c) * 64 + lane; };
    if (src) {
#pragma unroll
        for (int r = -1; r <= TY + 1; ++r) {
            if (slot[O + r] >= 0) {
                const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) amp_lds[lds_at(r, c)] = ld2(a, c);
            }
        }
    }
    const float2 tE0 = src ? ldc2(p.tE, n) : make_float2(0.f, 0.f);
    const float2 tE1 = src ? ldc2(p.tE, n + 1) : make_float2(0.f, 0.f);
    const float2 tH0 = src ? ldc2(p.tH, n) : make_float2(0.f, 0.f);
    const float2 tH1 = src ? ldc2(p.tH, n + 1) : make_float2(0.f, 0.f);
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
            if (!hold_x) pyx = a;
            if (!hold_x && !hy0) pzx = b2;
            tx_hz = stretched(ex_c.k, d_xhz, pyx);
            tx_hy = stretched(ex_c.k, d_xhy, pzx);
        }
        if constexpr (YB) {
            if (ysl(r) >= 0) {
                const Coef cy = eyc[O + r];
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
            pyx = cpml_mem(hx_c.b, pyx, hx_c.c, d_xez);
            pzx = cpml_mem(hx_c.b, pzx, hx_c.c, d_xey);
            tx_ez = stretched(hx_c.k, d_xez, pyx);
            tx_ey = stretched(hx_c.k, d_xey, pzx);
        }
        if constexpr (YB) {
            if (ysl(r) >= 0) {
                const Coef cy = hyc[O + r];
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

    // carried planes: H^{n+1/2}(q-1), E^{n+1}(q-1), H^{n+3/2}(q-2), E^{n+2}(q-2)
    float hpx[TY + 4], hpy[TY + 4], hpz[TY + 4];
    float e1x[TY + 4], e1y[TY + 4], e1z[TY + 4];
    float h1x[TY + 4], h1y[TY + 4], h1z[TY + 4];
    float e2x[TY + 4], e2y[TY + 4], e2z[TY + 4];
    // carried CPML memories: ψ_E^{n+1}(q-1) and ψ_H^{n+3/2}(q-2)
    constexpr int PX = XB ? TY + 4 : 1, PY = YB ? TY + 4 : 1;
    float qe_yx[PX], qe_zx[PX], qh_yx[PX], qh_zx[PX];
    float qe_xy[PY], qe_zy[PY], qh_xy[PY], qh_zy[PY];
#pragma unroll
    for (int r = 0; r < TY + 4; ++r) {
        hpx[r] = hpy[r] = hpz[r] = 0.f;
        e1x[r] = e1y[r] = e1z[r] = 0.f;
        h1x[r] = h1y[r] = h1z[r] = 0.f;
        e2x[r] = e2y[r] = e2z[r] = 0.f;
    }
#pragma unroll
    for (int r = 0; r < PX; ++r) qe_yx[r] = qe_zx[r] = qh_yx[r] = qh_zx[r] = 0.f;
#pragma unroll
    for (int r = 0; r < PY; ++r) qe_xy[r] = qe_zy[r] = qh_xy[r] = qh_zy[r] = 0.f;
    float dummy = 0.f;
    auto RX = [&](float* a, int r) -> float& {
        if constexpr (XB) return a[O + r];
        return dummy;
    };
    auto RY = [&](float* a, int r) -> float& {
        if constexpr (YB) return a[O + r];
        return dummy;
    };

    int kq = kb - 2;
    while (kq < 0) kq += nz;
    kq %= nz;
    int kq1 = 0, kq2 = 0;   // planes of q-1, q-2
    // e^{iβz} of planes q-1 and q-2 (integer, half plane), carried
    float2 za0 = make_float2(0.f, 0.f), za1 = za0, zb0 = za0, zb1 = za0;
    // interior tiles: the next plane's H rows are loaded at the end of a
    // plane, beside its stores
    constexpr bool PF = !XB && !YB;
    float nhx[TY + 4], nhy[TY + 4], nhz[TY + 4];
    if constexpr (PF) {
#pragma unroll
        for (int r = -2; r <= TY + 1; ++r) {
            nhx[O + r] = ld(HX, kq, r);
            nhz[O + r] = ld(HZ, kq, r);
            if (r >= -1) nhy[O + r] = ld(HY, kq, r);
        }
    }
    for (int q = kb - 2; q <= ke + 1; ++q) {
        // The four wavefronts of the workgroup start each plane together, so
        // the halo rows one loads are the rows its neighbour loads in the
        // same window (every wavefront passes this barrier equally often).
        __syncthreads();
        // ---- plane q of E^n and H^{n+1/2} --------------------------------
        float hx[TY + 4], hy[TY + 4], hz[TY + 4], ex[TY + 4], ey[TY + 4], ez[TY + 4];
#pragma unroll
        for (int r = -2; r <= TY + 1; ++r) {
            hx[O + r] = PF ? nhx[O + r] : ld(HX, kq, r);
            hz[O + r] = PF ? nhz[O + r] : ld(HZ, kq, r);
            if (r >= -1) {
                hy[O + r] = PF ? nhy[O + r] : ld(HY, kq, r);
                ex[O + r] = ld(EX, kq, r);
                ez[O + r] = ld(EZ, kq, r);
            }
            if (r >= -1 && r <= TY) ey[O + r] = ld(EY, kq, r);
        }
        float2 zq0 = make_float2(0.f, 0.f), zq1 = zq0;   // e^{iβz} of plane q
        if (src) {
            zq0 = ldc2(p.zph, 2 * kq);
            zq1 = ldc2(p.zph, 2 * kq + 1);
        }
        // CPML memories of both stages, issued with the field loads
        float pe_yx[PX], pe_zx[PX], pe_xy[PY], pe_zy[PY];   // ψ_E^n(q)
        float ph_yx[PX], ph_zx[PX], ph_xy[PY], ph_zy[PY];   // ψ_H^{n+1/2}(q-1)
#pragma unroll
        for (int r = -1; r <= TY + 1; ++r) {
            if constexpr (XB) {
                pe_yx[O + r] = r <= TY ? ldx(P_EYX, kq, r) : 0.f;
                pe_zx[O + r] = ldx(P_EZX, kq, r);
                if (r <= TY) {
                    ph_yx[O + r] = r >= 0 ? ldx(P_HYX, kq1, r) : 0.f;
                    ph_zx[O + r] = ldx(P_HZX, kq1, r);
                }
            }
            if constexpr (YB) {
                pe_xy[O + r] = ldy(P_EXY, kq, r);
                pe_zy[O + r] = ldy(P_EZY, kq, r);
                if (r <= TY) {
                    ph_xy[O + r] = ldy(P_HXY, kq1, r);
                    ph_zy[O + r] = ldy(P_HZY, kq1, r);
                }
            }
        }

        // ---- E^{n+1}(q), rows -1 .. TY+1 (E_y to TY), in place ------------
        {
            float2 pt0, pt1;
            phase(zq0, zq1, tE0, pt0, pt1);
#pragma unroll
            for (int r = -1; r <= TY + 1; ++r) {
                if (r > TY) ey[O + r] = 0.f;   // E_y is not formed on the last row
                const float hz_im = from_lower(hz[O + r]);
                const float hy_im = from_lower(hy[O + r]);
                e_upd(r, ex[O + r], ey[O + r], ez[O + r], hz[O + r] - hz[O + r - 1],
                      hy[O + r] - hpy[O + r], r <= TY ? hx[O + r] - hpx[O + r] : 0.f,
                      r <= TY ? hz[O + r] - hz_im : 0.f, hy[O + r] - hy_im,
                      hx[O + r] - hx[O + r - 1], RX(pe_yx, r), RX(pe_zx, r), RY(pe_xy, r),
                      RY(pe_zy, r), r <= TY);
                if (slot[O + r] >= 0) {
                    ex[O + r] += cmul_re(amp_lds[lds_at(r, EX)], pt0);
                    ez[O + r] += cmul_re(amp_lds[lds_at(r, EZ)], pt1);
                    if (r <= TY) ey[O + r] += cmul_re(amp_lds[lds_at(r, EY)], pt0);
                }
                zero_out(r, ex[O + r], ey[O + r], ez[O + r]);
            }
        }
        if (mask0 && kq == p.plane && q >= kb && q < ke && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r)
                if (row_st(r)) accumulate(mask0, r, ex[O + r], ey[O + r], ez[O + r]);
        }

        // ---- H^{n+3/2}(q-1), rows -1 .. TY (H_y from 0) --------------------
        float gx[TY + 4], gy[TY + 4], gz[TY + 4];
        {
            float2 qt0, qt1;
            phase(za0, za1, tH0, qt0, qt1);
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                const float ey_ip = from_upper(e1y[O + r]);
                const float ez_ip = from_upper(e1z[O + r]);
                gx[O + r] = hpx[O + r];
                gy[O + r] = r >= 0 ? hpy[O + r] : 0.f;
                gz[O + r] = hpz[O + r];
                h_upd(r, gx[O + r], gy[O + r], gz[O + r], e1z[O + r + 1] - e1z[O + r],
                      ey[O + r] - e1y[O + r], ex[O + r] - e1x[O + r], ez_ip - e1z[O + r],
                      ey_ip - e1y[O + r], e1x[O + r + 1] - e1x[O + r], RX(ph_yx, r),
                      RX(ph_zx, r), RY(ph_xy, r), RY(ph_zy, r), r >= 0);
                if (slot[O + r] >= 0) {
                    gx[O + r] += cmul_re(amp_lds[lds_at(r, HX)], qt1);
                    if (r >= 0) gy[O + r] += cmul_re(amp_lds[lds_at(r, HY)], qt1);
                    gz[O + r] += cmul_re(amp_lds[lds_at(r, HZ)], qt0);
                }
            }
        }

        // ---- E^{n+2}(q-1), rows 0 .. TY (E_y to TY-1) ----------------------
        float fx[TY + 4], fy[TY + 4], fz[TY + 4];
        const bool st1 = q - 1 >= kb && q - 1 < ke;
        {
            float2 pt0, pt1;
            phase(za0, za1, tE1, pt0, pt1);
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                const float hz_im = from_lower(gz[O + r]);
                const float hy_im = from_lower(gy[O + r]);
                fx[O + r] = e1x[O + r];
                fy[O + r] = r < TY ? e1y[O + r] : 0.f;
                fz[O + r] = e1z[O + r];
                e_upd(r, fx[O + r], fy[O + r], fz[O + r], gz[O + r] - gz[O + r - 1],
                      gy[O + r] - h1y[O + r], r < TY ? gx[O + r] - h1x[O + r] : 0.f,
                      r < TY ? gz[O + r] - hz_im : 0.f, gy[O + r] - hy_im,
                      gx[O + r] - gx[O + r - 1], RX(qe_yx, r), RX(qe_zx, r), RY(qe_xy, r),
                      RY(qe_zy, r), r < TY);
                if (slot[O + r] >= 0) {
                    fx[O + r] += cmul_re(amp_lds[lds_at(r, EX)], pt0);
                    fz[O + r] += cmul_re(amp_lds[lds_at(r, EZ)], pt1);
                    if (r < TY) fy[O + r] += cmul_re(amp_lds[lds_at(r, EY)], pt0);
                }
                zero_out(r, fx[O + r], fy[O + r], fz[O + r]);
            }
        }
        if (st1 && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (!row_st(r)) continue;
                st(EX, kq1, r, fx[O + r]);
                st(EY, kq1, r, fy[O + r]);
                st(EZ, kq1, r, fz[O + r]);
                if constexpr (XB) {
                    if (xsl >= 0) {
                        stx(P_EYX, kq1, r, qe_yx[O + r]);
                        stx(P_EZX, kq1, r, qe_zx[O + r]);
                    }
                }
                if constexpr (YB) {
                    if (ysl(r) >= 0) {
                        sty(P_EXY, kq1, r, qe_xy[O + r]);
                        sty(P_EZY, kq1, r, qe_zy[O + r]);
                    }
                }
            }
            if (mask1 && kq1 == p.plane) {
#pragma unroll
                for (int r = 0; r < TY; ++r)
                    if (row_st(r)) accumulate(mask1, r, fx[O + r], fy[O + r], fz[O + r]);
            }
        }

        // ---- H^{n+5/2}(q-2), rows 0 .. TY-1 --------------------------------
        if (q - 2 >= kb && q - 2 < ke) {
            float2 qt0, qt1;
            phase(zb0, zb1, tH1, qt0, qt1);
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const float ey_ip = from_upper(e2y[O + r]);
                const float ez_ip = from_upper(e2z[O + r]);
                float vx = h1x[O + r], vy = h1y[O + r], vz = h1z[O + r];
                h_upd(r, vx, vy, vz, e2z[O + r + 1] - e2z[O + r], fy[O + r] - e2y[O + r],
                      fx[O + r] - e2x[O + r], ez_ip - e2z[O + r], ey_ip - e2y[O + r],
                      e2x[O + r + 1] - e2x[O + r], RX(qh_yx, r), RX(qh_zx, r), RY(qh_xy, r),
                      RY(qh_zy, r), true);
                if (slot[O + r] >= 0) {
                    vx += cmul_re(amp_lds[lds_at(r, HX)], qt1);
                    vy += cmul_re(amp_lds[lds_at(r, HY)], qt1);
                    vz += cmul_re(amp_lds[lds_at(r, HZ)], qt0);
                }
                if (own && row_st(r)) {
                    st(HX, kq2, r, vx);
                    st(HY, kq2, r, vy);
                    st(HZ, kq2, r, vz);
                    if constexpr (XB) {
                        if (xsl >= 0) {
                            stx(P_HYX, kq2, r, qh_yx[O + r]);
                            stx(P_HZX, kq2, r, qh_zx[O + r]);
                        }
                    }
                    if constexpr (YB) {
                        if (ysl(r) >= 0) {
                            sty(P_HXY, kq2, r, qh_xy[O + r]);
                            sty(P_HZY, kq2, r, qh_zy[O + r]);
                        }
                    }
                }
            }
        }

        // ---- rotate ----------------------------------------------------------
#pragma unroll
        for (int r = -1; r <= TY + 1; ++r) {
            hpy[O + r] = hy[O + r];
            e1x[O + r] = ex[O + r];
            e1z[O + r] = ez[O + r];
            if (r <= TY) {
                hpx[O + r] = hx[O + r];
                hpz[O + r] = hz[O + r];
                e1y[O + r] = ey[O + r];
            }
        }
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            h1y[O + r] = gy[O + r];
            e2x[O + r] = fx[O + r];
            e2z[O + r] = fz[O + r];
            if (r < TY) {
                h1x[O + r] = gx[O + r];
                h1z[O + r] = gz[O + r];
                e2y[O + r] = fy[O + r];
            }
            if constexpr (XB) {
                qe_yx[O + r] = pe_yx[O + r];
                qe_zx[O + r] = pe_zx[O + r];
                qh_yx[O + r] = ph_yx[O + r];
                qh_zx[O + r] = ph_zx[O + r];
            }
            if constexpr (YB) {
                qe_xy[O + r] = pe_xy[O + r];
                qe_zy[O + r] = pe_zy[O + r];
                qh_xy[O + r] = ph_xy[O + r];
                qh_zy[O + r] = ph_zy[O + r];
            }
        }
        zb0 = za0;
        zb1 = za1;
        za0 = zq0;
        za1 = zq1;
        kq2 = kq1;
        kq1 = kq;
        kq = kq + 1 == nz ? 0 : kq + 1;
        if constexpr (PF) {
#pragma unroll
            for (int r = -2; r <= TY + 1; ++r) {
                nhx[O + r] = ld(HX, kq, r);
                nhz[O + r] = ld(HZ, kq, r);
                if (r >= -1) nhy[O + r] = ld(HY, kq, r);
            }
        }
    }
}

// Single domain: block b runs on XCD b % 8; blocks are remapped so that
// each XCD takes a contiguous run of tiles (consecutive segments of a row
// group and z chunk share halo rows in that XCD's L2).
template <int TY, bool XB, bool YB>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(step2_waves<TY, XB, YB>())))
step2_kernel(Problem p, long long n, int par, Launch2 L, int nblocks_padded, int mask0,
             int mask1) {
    const int nsl = span_count(L.seg), ngl = span_count(L.grp);
    const int ntile = nsl * ngl;
    const int lb = (blockIdx.x % 8) * (nblocks_padded / 8) + blockIdx.x / 8;
    if (lb >= ntile * L.ncz) return;
    const int t = lb % ntile;
    const int kb = (lb / ntile) * L.cz;
    step2_tile<TY, XB, YB>(p, n, par, span_at(L.seg, t % nsl), span_at(L.grp, t / nsl), kb,
                           min(kb + L.cz, p.nz), mask0, mask1);
}

// Many instances: one work item per workgroup, (instance, segment, row
// group, kb | ke << 16), all items of one tile class; the step index comes
// from a device counter (plus a launch offset) so that a captured graph
// stays valid when replayed.
template <int TY, bool XB, bool YB>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(step2_waves<TY, XB, YB>())))
step2_batch_kernel(const Problem* __restrict__ probs, const int4* __restrict__ items,
                   int nitems, int nblocks_padded, const long long* __restrict__ nctr, int off,
                   int par, int diag) {
    const int lb = (blockIdx.x % 8) * (nblocks_padded / 8) + blockIdx.x / 8;
    if (lb >= nitems) return;
    // the item is the same for the whole workgroup: keep it, and so the
    // Problem read with it, in scalar registers
    const int4 it = items[lb];
    const int q = __builtin_amdgcn_readfirstlane(it.x);
    const int seg = __builtin_amdgcn_readfirstlane(it.y);
    const int grp = __builtin_amdgcn_readfirstlane(it.z);
    const int kz = __builtin_amdgcn_readfirstlane(it.w);
    // read in place (restrict: no store of the kernel aliases it); a private
    // copy indexed by the runtime parity would leave scalar registers
    const Problem& p = probs[q];
    const long long n = *nctr + off;
    const int m0 = diag && p.plane >= 0 && n >= p.win_begin ? p.diag_mask : 0;
    const int m1 = diag && p.plane >= 0 && n + 1 >= p.win_begin ? p.diag_mask : 0;
    step2_tile<TY, XB, YB>(p, n, par, seg, grp, kz & 0xffff, kz >> 16, m0, m1);
}

// LDS of the staged antenna amplitudes of one workgroup: the 4 TY + 3 rows
// its wavefronts form, six components, 64 lanes (33 KiB at TY = 2).
constexpr unsigned amp_lds_bytes(int ty) {
    return (unsigned)((WAVES * ty + 3) * 6 * 64 * sizeof(float2));
}

// Segments and row groups whose tiles form only regular cells (an interval
// each, possibly empty).
struct Plan2 {
    int nseg, ngrp, s_lo, s_hi, g_lo, g_hi, cz, ncz;
};

Plan2 plan2(const Problem& p, int rows, int zchunk) {
    Plan2 P{};
    const int G = WAVES * rows;
    P.nseg = (p.nx + OWN - 1) / OWN;
    P.ngrp = (p.ny + G - 1) / G;
    const int m = std::max(p.npml, 1);
    // segment s: lanes x = 60 s - 2 + l; lanes 1..63 must be regular cells,
    // lane 0 inside the grid
    P.s_lo = P.nseg;
    P.s_hi = P.nseg;
    for (int s = 0; s < P.nseg; ++s) {
        const int x0 = OWN * s - 2;
        const bool reg = x0 >= 0 && x0 + 1 >= m && x0 + 63 <= p.nx - p.npml - 1;
        if (reg && P.s_lo == P.nseg) P.s_lo = s;
        if (reg) P.s_hi = s + 1;
    }
    if (P.s_lo >= P.s_hi) P.s_lo = P.s_hi = P.nseg;
    // row group g: formed rows g G - 1 .. g G + G + 1 regular (row g G - 2 is
    // only read)
    P.g_lo = P.ngrp;
    P.g_hi = P.ngrp;
    for (int g = 0; g < P.ngrp; ++g) {
        const bool reg = g * G - 1 >= m && g * G + G + 1 <= p.ny - p.npml - 1;
        if (reg && P.g_lo == P.ngrp) P.g_lo = g;
        if (reg) P.g_hi = g + 1;
    }
    if (P.g_lo >= P.g_hi) P.g_lo = P.g_hi = P.ngrp;
    P.cz = zchunk > 0 ? std::min(zchunk, p.nz) : p.nz;
    P.ncz = (p.nz + P.cz - 1) / P.cz;
    return P;
}

template <int TY, bool XB, bool YB>
hipError_t launch_class(const Problem& p, long long n, int parity, const Launch2& L, int mask0,
                        int mask1, hipStream_t s, LaunchTimer* timer, const char* name) {
    const int nt = span_count(L.seg) * span_count(L.grp) * L.ncz;
    if (nt <= 0) return hipSuccess;
    const int nbp = (nt + 7) / 8 * 8;
    if (timer) timer->mark_on(name, s);
    hipLaunchKernelGGL((step2_kernel<TY, XB, YB>), dim3(nbp), dim3(64 * WAVES),
                       p.colmap ? amp_lds_bytes(TY) : 0, s, p, n,
                       parity, L, nbp, mask0, mask1);
    hipError_t e = hipGetLastError();
    if (timer) timer->mark_on(nullptr, s);
    return e;
}

// The four classes touch disjoint cells: with side streams the boundary
// classes run beside the interior launch, forked from and joined back into
// s by events (a per-launch timer brackets each kernel on its own stream).
template <int TY>
hipError_t launch_rows(const Problem& p, long long n, int parity, int zchunk, int mask0,
                       int mask1, hipStream_t s, LaunchTimer* timer, const SideStreams* side) {
    const Plan2 P = plan2(p, TY, zchunk);
    const Span s_int{P.s_lo, P.s_hi, 0, 0}, s_bnd{0, P.s_lo, P.s_hi, P.nseg};
    const Span g_int{P.g_lo, P.g_hi, 0, 0}, g_bnd{0, P.g_lo, P.g_hi, P.ngrp};
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
    // give them more workgroups (and a shorter critical path) at the cost
    // of re-reading two planes at each chunk end.
    const int czc = std::min(P.cz, 8), czy = std::min(P.cz, 16);
    e = launch_class<TY, true, true>(p, n, parity,
                                     Launch2{s_bnd, g_bnd, czc, (p.nz + czc - 1) / czc}, mask0,
                                     mask1, sc, timer, "step2_corner");
    if (e == hipSuccess)
        e = launch_class<TY, false, true>(p, n, parity,
                                          Launch2{s_int, g_bnd, czy, (p.nz + czy - 1) / czy},
                                          mask0, mask1, sy, timer, "step2_ybnd");
    if (e == hipSuccess)
        e = launch_class<TY, true, false>(p, n, parity, Launch2{s_bnd, g_int, P.cz, P.ncz}, mask0,
                                          mask1, sx, timer, "step2_xbnd");
    if (e == hipSuccess)
        e = launch_class<TY, false, false>(p, n, parity, Launch2{s_int, g_int, P.cz, P.ncz}, mask0,
                                           mask1, s, timer, "step2_interior");
    if (fork) {
        for (int q = 0; q < 3; ++q) {
            hipError_t f = hipEventRecord(side->join[q], side->s[q]);
            if (f == hipSuccess) f = hipStreamWaitEvent(s, side->join[q], 0);
            if (e == hipSuccess) e = f;
        }
    }
    return e;
}

template <int TY, bool XB, bool YB>
hipError_t launch_batch_class(const Problem* probs, const int4* items, int nitems,
                              const long long* nctr, int off, int par, int diag, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int nbp = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((step2_batch_kernel<TY, XB, YB>), dim3(nbp), dim3(64 * WAVES),
                       amp_lds_bytes(TY), s,
                       probs, items, nitems, nbp, nctr, off, par, diag);
    return hipGetLastError();
}

template <int TY>
hipError_t launch_batch_rows(const Problem* probs, const int4* const items[4],
                             const int nitems[4], const long long* nctr, int off, int par,
                             int diag, hipStream_t s, const SideStreams* side) {
    hipStream_t sx = s, sy = s, sc = s;
    hipError_t e = hipSuccess;
    if (side) {
        e = hipEventRecord(side->fork, s);
        for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipStreamWaitEvent(side->s[q], side->fork, 0);
        if (e != hipSuccess) return e;
        sx = side->s[0];
        sy = side->s[1];
        sc = side->s[2];
    }
    e = launch_batch_class<TY, true, true>(probs, items[3], nitems[3], nctr, off, par, diag, sc);
    if (e == hipSuccess)
        e = launch_batch_class<TY, false, true>(probs, items[2], nitems[2], nctr, off, par, diag,
                                                sy);
    if (e == hipSuccess)
        e = launch_batch_class<TY, true, false>(probs, items[1], nitems[1], nctr, off, par, diag,
                                                sx);
    if (e == hipSuccess)
        e = launch_batch_class<TY, false, false>(probs, items[0], nitems[0], nctr, off, par,
                                                 diag, s);
    if (side) {
        for (int q = 0; q < 3; ++q) {
            hipError_t f = hipEventRecord(side->join[q], side->s[q]);
            if (f == hipSuccess) f = hipStreamWaitEvent(s, side->join[q], 0);
            if (e == hipSuccess) e = f;
        }
    }
    return e;
}

}  // namespace

long long step2_interior_cells(const Problem& p, int rows) {
    const Plan2 P = plan2(p, rows, 0);
    if (P.s_lo >= P.s_hi || P.g_lo >= P.g_hi) return 0;
    const long long xs = std::min(OWN * P.s_hi, p.nx) - OWN * P.s_lo;
    const long long ys = std::min(WAVES * rows * P.g_hi, p.ny) - WAVES * rows * P.g_lo;
    return xs * ys * p.nz;
}

hipError_t launch_step2(const Problem& p, long long n, int parity, int rows, int zchunk,
                        int mask0, int mask1, hipStream_t s, LaunchTimer* timer,
                        const SideStreams* side) {
    if (p.periodic) return hipErrorInvalidValue;
    if (rows == 2) return launch_rows<2>(p, n, parity, zchunk, mask0, mask1, s, timer, side);
    if (rows == 4) return launch_rows<4>(p, n, parity, zchunk, mask0, mask1, s, timer, side);
    return hipErrorInvalidValue;
}

void step2_batch_items(const std::vector<Problem>& probs, int rows, int zchunk,
                       std::vector<int4> items[4]) {
    for (int c = 0; c < 4; ++c) items[c].clear();
    for (int q = 0; q < (int)probs.size(); ++q) {
        const Problem& p = probs[q];
        const Plan2 P = plan2(p, rows, zchunk);
        for (int ch = 0; ch < P.ncz; ++ch) {
            const int kb = ch * P.cz, ke = std::min(kb + P.cz, p.nz);
            for (int g = 0; g < P.ngrp; ++g) {
                const bool gi = g >= P.g_lo && g < P.g_hi;
                for (int sg = 0; sg < P.nseg; ++sg) {
                    const bool si = sg >= P.s_lo && sg < P.s_hi;
                    const int cls = (si ? 0 : 1) + (gi ? 0 : 2);
                    items[cls].push_back(make_int4(q, sg, g, kb | (ke << 16)));
                }
            }
        }
    }
}

hipError_t launch_step2_batch(const Problem* probs, const int4* const items[4],
                              const int nitems[4], int rows, const long long* nctr, int off,
                              int par, int diag, hipStream_t s, const SideStreams* side) {
    if (rows == 2)
        return launch_batch_rows<2>(probs, items, nitems, nctr, off, par, diag, s, side);
    if (rows == 4)
        return launch_batch_rows<4>(probs, items, nitems, nctr, off, par, diag, s, side);
    return hipErrorInvalidValue;
}

}  // namespace bfdtd
