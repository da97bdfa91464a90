// Two-step fused interior kernel (temporal blocking): one pass over the
// fields advances the interior by two leapfrog steps, E^n, H^{n+1/2} ->
// E^{n+2}, H^{n+5/2}, reading the old ping-pong buffers once and writing
// the new ones once: 48 B of field traffic per cell for two cell-updates.
// Each cell is computed with the same expressions, in the same order, as the
// one-step kernels (kernels_fused.hip, yee_cell.hpp), so the result is
// bit-identical to two one-step launches.
//
// Work decomposition (CDNA4, wave64). A wavefront reads a block of 64 x
// cells (lane l at x = x0 - 2 + l) × TY + 4 rows (j0 - 2 .. j0 + TY + 1) and
// marches along z. The intermediate step is formed in registers on every
// lane and every row it can be formed on, so the second step needs nothing
// from other wavefronts:
//   x: neighbours move between lanes with DPP wavefront shifts; lanes 0-1
//      and 62-63 are halo, the wavefront stores at most lanes 2..61 (60
//      cells), and the tiles advance by 60 cells.
//   y: E^{n+1} is formed on rows -1 .. TY+1, H^{n+3/2} on rows -1 .. TY,
//      E^{n+2} on rows 0 .. TY, H^{n+5/2} on the TY stored rows.
//   z: at plane q the pipeline forms E^{n+1}(q), H^{n+3/2}(q-1),
//      E^{n+2}(q-1) and H^{n+5/2}(q-2), keeping one plane of each in
//      registers; a chunk [kb, ke) reads planes kb-2 .. ke+1 (z is periodic).
//      A workgroup stacks four wavefronts in y that start every plane
//      together (one barrier per plane).
// The cells a wavefront forms must all be regular (no wall, no CPML), which
// bounds the interior to x0 - 1, j0 - 1 >= m + 1 and x0 + 61, j0 + TY + 1 <=
// n - npml - 1. The frame around it is advanced by the split kernels in
// four passes through an intermediate buffer (context.hpp); the kernel
// writes into that buffer the intermediate values of its edge cells that
// those passes read.
//
// Addresses: a wave-uniform 64-bit base (component, plane, row, tile
// origin) in scalar registers plus the lane's byte offset, so every size
// takes the same path.
#include <hip/hip_runtime.h>

#include <algorithm>

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

struct Interior2 {
    int x_org, x_end, y_org, nseg, nrow, ncz, cz;
};

// x: [x_org, x_end) on 32-cell (128-byte) boundaries, so that the frame's x
// strips are whole lines; tiles of 60 cells from x_org, the last one shifted
// left to end at x_end (it stores only the cells the others leave).
// Every cell a wavefront forms lies in [m + 1, n - npml - 1] in x and y.
Interior2 interior2(const Problem& p, int rows, int zchunk) {
    Interior2 I{0, 0, 0, 0, 0, 0, 0};
    if (p.periodic) return I;
    const int m = p.npml > 0 ? p.npml : 1;
    const int hi_x = p.nx - p.npml - 1, hi_y = p.ny - p.npml - 1;
    I.x_org = (m + 2 + 31) / 32 * 32;
    I.x_end = (hi_x - 1) / 32 * 32;
    I.y_org = m + 2;
    const int sy = hi_y - (rows + 1) - I.y_org;
    I.nseg = I.x_end - I.x_org >= OWN ? (I.x_end - I.x_org + OWN - 1) / OWN : 0;
    I.nrow = sy >= 0 ? sy / rows + 1 : 0;
    I.cz = zchunk > 0 ? std::min(zchunk, p.nz) : p.nz;
    I.ncz = (p.nz + I.cz - 1) / I.cz;
    if (I.nseg <= 0 || I.nrow <= 0) I.nseg = I.nrow = 0;
    return I;
}

int group_count2(const Interior2& I) {
    return I.nseg * ((I.nrow + WAVES - 1) / WAVES) * I.ncz;
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

template <int TY>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(TY == 2 ? 3 : 2)))
fused2_interior_kernel(Problem p, long long n, int par, Interior2 I, int nblocks_padded,
                       int mask0, int mask1, float* mid) {
    // ---- which tile: hardware block b runs on XCD b % 8 ----------------
    const int nrq = (I.nrow + WAVES - 1) / WAVES;
    const int lb = (blockIdx.x % 8) * (nblocks_padded / 8) + blockIdx.x / 8;
    if (lb >= I.nseg * nrq * I.ncz) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int seg = lb % I.nseg;
    const int sy = ((lb / I.nseg) % nrq) * WAVES + w;
    const int kb = (lb / (I.nseg * nrq)) * I.cz;
    const int ke = min(kb + I.cz, p.nz);
    if (sy >= I.nrow) {                                        // uniform per wavefront
        for (int q = kb - 2; q <= ke + 1; ++q) __syncthreads(); // the others' barriers
        return;
    }
    const int lane = threadIdx.x & 63;
    const int j0 = I.y_org + sy * TY;
    const bool last = seg == I.nseg - 1;
    const int own_lo = I.x_org + OWN * seg;                    // stored x range
    const int own_hi = last ? I.x_end : own_lo + OWN;
    const int xs = last ? I.x_end - OWN - 2 : own_lo - 2;      // x of lane 0
    const int x = xs + lane;
    const bool own = x >= own_lo && x < own_hi;
    // cells on the rectangle's edge whose intermediate values the frame
    // passes read: E^{n+1} on the low-x / low-y edge, H^{n+3/2} on the
    // high-x / high-y edge (uniform test first: most tiles have none)
    const int y_end = I.y_org + TY * I.nrow;
    const bool edge_lo = seg == 0 || sy == 0;
    const bool edge_hi = last || sy == I.nrow - 1;
    const int nz = p.nz, nx = p.nx, ny = p.ny;
    const size_t plane = (size_t)ny * p.pitch;
    const gptr<const float> fo = G((const float*)p.fbase[par]);
    const gptr<float> fw = G(p.fbase[par ^ 1]);
    const size_t fs = (size_t)p.fstride;
    // element offset of (component c, plane kk, row r) at lane 0: uniform
    auto base = [&](int c, int kk, int r) {
        return (size_t)c * fs + (size_t)kk * plane + (size_t)(j0 + r) * p.pitch + xs;
    };
    // The uniform address (component, plane, row, tile) is formed in scalar
    // registers; each access adds the lane's byte offset to it. (Buffer
    // instructions with a scalar descriptor save that add but measured
    // slower here.)
    const unsigned lo4 = 4u * (unsigned)lane;
    auto ld = [&](int c, int kk, int r) {
        return *(gptr<const float>)(uniform(fo + base(c, kk, r)) + lo4);
    };
    // plain stores: a tile stores 60 cells of a row, so lines at tile edges
    // are written by two tiles and merge in L2
    auto st = [&](int c, int kk, int r, float v) {
        *(gptr<float>)(uniform(fw + base(c, kk, r)) + lo4) = v;
    };
    const gptr<float> fm = G(mid);
    auto st_mid = [&](int c, int kk, int r, float v) {
        *(gptr<float>)(uniform(fm + base(c, kk, r)) + lo4) = v;
    };

    const bool src = p.colmap != nullptr;
    int slot[TY + 4];
#pragma unroll
    for (int r = -1; r <= TY + 1; ++r)
        slot[O + r] = src ? G(p.colmap)[(size_t)(j0 + r) * nx + x] : -1;
    const gptr<const float2> amp = G(p.amp);
    const float2 tE0 = src ? ld2(G(p.tE), n) : make_float2(0.f, 0.f);
    const float2 tE1 = src ? ld2(G(p.tE), n + 1) : make_float2(0.f, 0.f);
    const float2 tH0 = src ? ld2(G(p.tH), n) : make_float2(0.f, 0.f);
    const float2 tH1 = src ? ld2(G(p.tH), n + 1) : make_float2(0.f, 0.f);
    // e^{iβz} at the integer / half planes of kk times a time factor
    auto phase = [&](int kk, float2 t, float2& a0, float2& a1) {
        a0 = make_float2(0.f, 0.f);
        a1 = a0;
        if (src) {
            a0 = cmul(ld2(G(p.zph), 2 * kk), t);
            a1 = cmul(ld2(G(p.zph), 2 * kk + 1), t);
        }
    };
    const gptr<double> fl = G(p.fl);
    auto accumulate = [&](int mask, int r, float vx, float vy, float vz) {
        const size_t pl = (size_t)(j0 + r) * nx + x, ps = (size_t)nx * ny;
        if (mask & FDTD_DIAG_EX2) fl[pl] += (double)vx * vx;
        if (mask & FDTD_DIAG_EY2) fl[ps + pl] += (double)vy * vy;
        if (mask & FDTD_DIAG_EZ2) fl[2 * ps + pl] += (double)vz * vz;
    };

    // carried planes: H^{n+1/2}(q-1), E^{n+1}(q-1), H^{n+3/2}(q-2), E^{n+2}(q-2)
    float hpx[TY + 4], hpy[TY + 4], hpz[TY + 4];
    float e1x[TY + 4], e1y[TY + 4], e1z[TY + 4];
    float h1x[TY + 4], h1y[TY + 4], h1z[TY + 4];
    float e2x[TY + 4], e2y[TY + 4], e2z[TY + 4];
#pragma unroll
    for (int r = 0; r < TY + 4; ++r) {
        hpx[r] = hpy[r] = hpz[r] = 0.f;
        e1x[r] = e1y[r] = e1z[r] = 0.f;
        h1x[r] = h1y[r] = h1z[r] = 0.f;
        e2x[r] = e2y[r] = e2z[r] = 0.f;
    }

    int kq = kb - 2;
    while (kq < 0) kq += nz;
    kq %= nz;
    int kq1 = 0, kq2 = 0;   // planes of q-1, q-2
    for (int q = kb - 2; q <= ke + 1; ++q) {
        // The four wavefronts of the workgroup start each plane together, so
        // the halo rows one loads are the rows its neighbour loads in the
        // same window (every wavefront passes this barrier equally often).
        __syncthreads();
        // ---- plane q of E^n and H^{n+1/2} --------------------------------
        float hx[TY + 4], hy[TY + 4], hz[TY + 4], ex[TY + 4], ey[TY + 4], ez[TY + 4];
#pragma unroll
        for (int r = -2; r <= TY + 1; ++r) {
            hx[O + r] = ld(HX, kq, r);
            hz[O + r] = ld(HZ, kq, r);
            if (r >= -1) {
                hy[O + r] = ld(HY, kq, r);
                ex[O + r] = ld(EX, kq, r);
                ez[O + r] = ld(EZ, kq, r);
            }
            if (r >= -1 && r <= TY) ey[O + r] = ld(EY, kq, r);
        }

        // ---- E^{n+1}(q), rows -1 .. TY+1 (E_y to TY), in place ------------
        {
            float2 pt0, pt1;
            phase(kq, tE0, pt0, pt1);
#pragma unroll
            for (int r = -1; r <= TY + 1; ++r) {
                const float hz_im = from_lower(hz[O + r]);
                const float hy_im = from_lower(hy[O + r]);
                ex[O + r] += p.sy * (hz[O + r] - hz[O + r - 1]) - p.sz * (hy[O + r] - hpy[O + r]);
                ez[O + r] += p.sx * (hy[O + r] - hy_im) - p.sy * (hx[O + r] - hx[O + r - 1]);
                if (r <= TY)
                    ey[O + r] += p.sz * (hx[O + r] - hpx[O + r]) - p.sx * (hz[O + r] - hz_im);
                if (slot[O + r] >= 0) {
                    const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
                    ex[O + r] += cmul_re(ld2(a, EX), pt0);
                    ez[O + r] += cmul_re(ld2(a, EZ), pt1);
                    if (r <= TY) ey[O + r] += cmul_re(ld2(a, EY), pt0);
                }
            }
        }
        if (mask0 && kq == p.plane && q >= kb && q < ke && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r) accumulate(mask0, r, ex[O + r], ey[O + r], ez[O + r]);
        }
        if (edge_lo && q >= kb && q < ke) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (own && (x == I.x_org || j0 + r == I.y_org)) {
                    st_mid(EX, kq, r, ex[O + r]);
                    st_mid(EY, kq, r, ey[O + r]);
                    st_mid(EZ, kq, r, ez[O + r]);
                }
            }
        }

        // ---- H^{n+3/2}(q-1), rows -1 .. TY (H_y from 0) --------------------
        float gx[TY + 4], gy[TY + 4], gz[TY + 4];
        {
            float2 qt0, qt1;
            phase(kq1, tH0, qt0, qt1);
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                const float ey_ip = from_upper(e1y[O + r]);
                const float ez_ip = from_upper(e1z[O + r]);
                gx[O + r] = hpx[O + r] - (p.sy * (e1z[O + r + 1] - e1z[O + r]) -
                                          p.sz * (ey[O + r] - e1y[O + r]));
                if (r >= 0)
                    gy[O + r] = hpy[O + r] - (p.sz * (ex[O + r] - e1x[O + r]) -
                                              p.sx * (ez_ip - e1z[O + r]));
                gz[O + r] = hpz[O + r] - (p.sx * (ey_ip - e1y[O + r]) -
                                          p.sy * (e1x[O + r + 1] - e1x[O + r]));
                if (slot[O + r] >= 0) {
                    const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
                    gx[O + r] += cmul_re(ld2(a, HX), qt1);
                    if (r >= 0) gy[O + r] += cmul_re(ld2(a, HY), qt1);
                    gz[O + r] += cmul_re(ld2(a, HZ), qt0);
                }
            }
        }

        if (edge_hi && q - 1 >= kb && q - 1 < ke) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (own && (x == I.x_end - 1 || j0 + r == y_end - 1)) {
                    st_mid(HX, kq1, r, gx[O + r]);
                    st_mid(HY, kq1, r, gy[O + r]);
                    st_mid(HZ, kq1, r, gz[O + r]);
                }
            }
        }

        // ---- E^{n+2}(q-1), rows 0 .. TY (E_y to TY-1) ----------------------
        float fx[TY + 4], fy[TY + 4], fz[TY + 4];
        {
            float2 pt0, pt1;
            phase(kq1, tE1, pt0, pt1);
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                const float hz_im = from_lower(gz[O + r]);
                const float hy_im = from_lower(gy[O + r]);
                fx[O + r] = e1x[O + r];
                fz[O + r] = e1z[O + r];
                fx[O + r] += p.sy * (gz[O + r] - gz[O + r - 1]) - p.sz * (gy[O + r] - h1y[O + r]);
                fz[O + r] += p.sx * (gy[O + r] - hy_im) - p.sy * (gx[O + r] - gx[O + r - 1]);
                if (r < TY) {
                    fy[O + r] = e1y[O + r];
                    fy[O + r] += p.sz * (gx[O + r] - h1x[O + r]) - p.sx * (gz[O + r] - hz_im);
                }
                if (slot[O + r] >= 0) {
                    const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
                    fx[O + r] += cmul_re(ld2(a, EX), pt0);
                    fz[O + r] += cmul_re(ld2(a, EZ), pt1);
                    if (r < TY) fy[O + r] += cmul_re(ld2(a, EY), pt0);
                }
            }
        }
        const bool st1 = q - 1 >= kb && q - 1 < ke;
        if (st1 && own) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                st(EX, kq1, r, fx[O + r]);
                st(EY, kq1, r, fy[O + r]);
                st(EZ, kq1, r, fz[O + r]);
            }
            if (mask1 && kq1 == p.plane) {
#pragma unroll
                for (int r = 0; r < TY; ++r) accumulate(mask1, r, fx[O + r], fy[O + r], fz[O + r]);
            }
        }

        // ---- H^{n+5/2}(q-2), rows 0 .. TY-1 --------------------------------
        if (q - 2 >= kb && q - 2 < ke) {
            float2 qt0, qt1;
            phase(kq2, tH1, qt0, qt1);
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const float ey_ip = from_upper(e2y[O + r]);
                const float ez_ip = from_upper(e2z[O + r]);
                float vx = h1x[O + r] - (p.sy * (e2z[O + r + 1] - e2z[O + r]) -
                                         p.sz * (fy[O + r] - e2y[O + r]));
                float vy = h1y[O + r] - (p.sz * (fx[O + r] - e2x[O + r]) -
                                         p.sx * (ez_ip - e2z[O + r]));
                float vz = h1z[O + r] - (p.sx * (ey_ip - e2y[O + r]) -
                                         p.sy * (e2x[O + r + 1] - e2x[O + r]));
                if (slot[O + r] >= 0) {
                    const gptr<const float2> a = amp + (size_t)slot[O + r] * 6;
                    vx += cmul_re(ld2(a, HX), qt1);
                    vy += cmul_re(ld2(a, HY), qt1);
                    vz += cmul_re(ld2(a, HZ), qt0);
                }
                if (own) {
                    st(HX, kq2, r, vx);
                    st(HY, kq2, r, vy);
                    st(HZ, kq2, r, vz);
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
        }
        kq2 = kq1;
        kq1 = kq;
        kq = kq + 1 == nz ? 0 : kq + 1;
    }
}

template <int TY>
hipError_t launch_rows2(const Problem& p, long long n, int parity, int zchunk, int mask0,
                        int mask1, float* mid, hipStream_t s, LaunchTimer* timer) {
    const Interior2 I = interior2(p, TY, zchunk);
    const int nb = group_count2(I);
    if (nb <= 0) return hipSuccess;
    const int nbp = (nb + 7) / 8 * 8;
    if (timer) timer->mark("fused2_interior");
    hipLaunchKernelGGL((fused2_interior_kernel<TY>), dim3(nbp), dim3(64 * WAVES), 0, s, p, n,
                       parity, I, nbp, mask0, mask1, mid);
    hipError_t e = hipGetLastError();
    if (timer) timer->mark(nullptr);
    return e;
}

}  // namespace

Frame fused2_interior_rect(const Problem& p, int rows) {
    const Interior2 I = interior2(p, rows, 0);
    if (I.nseg <= 0) return Frame{0, 0, 0, 0};
    return Frame{I.x_org, I.x_end, I.y_org, I.y_org + rows * I.nrow};
}

hipError_t launch_fused2_interior(const Problem& p, long long n, int parity, int rows, int zchunk,
                                  int mask0, int mask1, float* mid, hipStream_t s,
                                  LaunchTimer* timer) {
    if (!mid) return hipErrorInvalidValue;
    if (rows == 2) return launch_rows2<2>(p, n, parity, zchunk, mask0, mask1, mid, s, timer);
    if (rows == 4) return launch_rows2<4>(p, n, parity, zchunk, mask0, mask1, mid, s, timer);
    return hipErrorInvalidValue;
}

}  // namespace bfdtd
