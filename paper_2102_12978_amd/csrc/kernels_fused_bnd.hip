// Fused Yee step for tiles that touch walls, CPML slabs or grid edges: the
// register-blocked z march of the interior kernel (E_new(k+1) from H_old(k+1)
// and H_old(k), then H_new(k) from E_new(k) and E_new(k+1), one read of the
// old fields and one write of the new ones), with every cell going through
// the per-cell boundary code of the split kernels (e_cell / h_cell: PEC
// holds, CPML memories, soft source), so a cell gets the same value as in a
// split-kernel step.
//
// A wavefront owns one tile: 64 x cells (x0 = 64 s) × TY rows (y0 = TY g),
// a chunk of z planes. Lanes past nx read the zero padding of the row pitch
// and are never stored; rows outside [0, ny) read as zero (the values beyond
// the PEC walls). A cell is stored only if it is inside the grid and outside
// the excluded rectangle (the part another kernel updates). The halo columns
// x0-1 and x0+64 come from one gather per plane; E_new at x0+64 is formed
// wavefront-uniform by the same per-cell code, without storing its CPML
// memories. Tiles come from a list (instance, x0, y0, z chunk) walked by a
// persistent grid; consecutive tiles are x-adjacent, so the four wavefronts
// of a workgroup share halo lines.
#include <hip/hip_runtime.h>

#include "yee_cell.hpp"

namespace bfdtd {

namespace {

constexpr int SEG = 64;
constexpr int WAVES = 4;

__device__ __forceinline__ float ldb(gptr<const float> base, unsigned boff) {
    return *(gptr<const float>)((gptr<const char>)base + boff);
}

__device__ __forceinline__ void stb(gptr<float> base, unsigned boff, float v) {
    __builtin_nontemporal_store(v, (gptr<float>)((gptr<char>)base + boff));
}

__device__ __forceinline__ float bcastb(float v, int q) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), q));
}

// Halo gather layout (value q of a plane is loaded by lane q).
template <int TY>
struct BHalo {
    static constexpr int R_HX = 0;              // x0+64: H_x rows -1..TY-1
    static constexpr int R_HY = TY + 1;         //        H_y rows 0..TY-1
    static constexpr int R_HZ = 2 * TY + 1;     //        H_z rows -1..TY-1
    static constexpr int R_EX = 3 * TY + 2;     //        E_x rows 0..TY-1
    static constexpr int R_EY = 4 * TY + 2;     //        E_y
    static constexpr int R_EZ = 5 * TY + 2;     //        E_z
    static constexpr int L_HY = 6 * TY + 2;     // x0-1:  H_y rows 0..TY
    static constexpr int L_HZ = 7 * TY + 3;     //        H_z rows 0..TY
    static constexpr int COUNT = 8 * TY + 4;
    static_assert(COUNT <= 64, "halo gather exceeds one wavefront");
};

// (component, row offset, column) of gather slot q; row offsets are relative
// to y0, the column is x0+64 or x0-1.
template <int TY>
__device__ __forceinline__ void bhalo_slot(int q, int x0, int* c, int* r, int* x) {
    using H = BHalo<TY>;
    *x = x0 + SEG;
    if (q >= H::L_HZ) { *c = HZ; *r = q - H::L_HZ; *x = x0 - 1; }
    else if (q >= H::L_HY) { *c = HY; *r = q - H::L_HY; *x = x0 - 1; }
    else if (q >= H::R_EZ) { *c = EZ; *r = q - H::R_EZ; }
    else if (q >= H::R_EY) { *c = EY; *r = q - H::R_EY; }
    else if (q >= H::R_EX) { *c = EX; *r = q - H::R_EX; }
    else if (q >= H::R_HZ) { *c = HZ; *r = q - H::R_HZ - 1; }
    else if (q >= H::R_HY) { *c = HY; *r = q - H::R_HY; }
    else { *c = HX; *r = q - 1; }
}

// MULTI: tiles of many instances (probs[instance]); otherwise of `single`.
// Two instantiations keep every Problem access in one address space (the
// kernel argument or global memory), so no generic pointer reaches the
// per-cell code.
template <int TY, bool MULTI>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(TY == 2 ? 3 : 2)))
fused_bnd_kernel(Problem single, const Problem* __restrict__ probs, const int4* __restrict__ tiles,
                 int ntiles, int cz, const long long* __restrict__ nctr, long long n_off, int par,
                 int diag, Frame excl, double* epart) {
    using H = BHalo<TY>;
    const long long n = (nctr ? *nctr : 0) + n_off;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int t = blockIdx.x * WAVES + w; t < ntiles; t += gridDim.x * WAVES) {
        const int4 tl = tiles[t];
        const Problem& p = MULTI ? probs[tl.x] : single;
        const int x0 = tl.y, j0 = tl.z;
        const int nx = p.nx, ny = p.ny, nz = p.nz;
        const int kb = tl.w * cz, ke = min(kb + cz, nz);
        const int x = x0 + lane;
        const bool xin = x < nx;
        const int mask = (diag && n >= p.win_begin) ? p.diag_mask : 0;
        const size_t plane = (size_t)ny * p.pitch;   // floats per plane
        gptr<const float> fo[6];
        gptr<float> fw[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            fo[c] = G(p.fbase[par]) + c * p.fstride;
            fw[c] = G(p.fbase[par ^ 1]) + c * p.fstride;
        }
        // rows y0-1 .. y0+TY: byte offset (clamped into the grid) and validity
        unsigned ro[TY + 2];
        bool rv[TY + 2];
#pragma unroll
        for (int r = -1; r <= TY; ++r) {
            const int y = j0 + r;
            rv[r + 1] = y >= 0 && y < ny;
            ro[r + 1] = 4u * (unsigned)(min(max(y, 0), ny - 1) * p.pitch + x);
        }
        auto ld = [&](int c, int kk, int r) -> float {
            const float v = ldb(fo[c] + (size_t)kk * plane, ro[r + 1]);
            return rv[r + 1] ? v : 0.f;
        };
        auto owned = [&](int r) -> bool {
            const int y = j0 + r;
            return xin && y < ny &&
                   !(x >= excl.x0 && x < excl.x1 && y >= excl.y0 && y < excl.y1);
        };
        int slot[TY + 1];
#pragma unroll
        for (int r = 0; r <= TY; ++r)
            slot[r] = (p.colmap && xin && rv[r + 1]) ? G(p.colmap)[(size_t)(j0 + r) * nx + x] : -1;
        // right halo column
        const bool hr = x0 + SEG < nx;              // E at x0+64 exists
        const bool hl = x0 > 0;                     // H at x0-1 exists
        int slot_h[TY];
#pragma unroll
        for (int r = 0; r < TY; ++r)
            slot_h[r] = (p.colmap && hr && j0 + r < ny) ? G(p.colmap)[(size_t)(j0 + r) * nx + x0 + SEG]
                                                        : -1;
        // gather slot of this lane
        gptr<const float> gp = fo[0];
        bool gv = false;
        if (lane < H::COUNT) {
            int c, r, gx;
            bhalo_slot<TY>(lane, x0, &c, &r, &gx);
            const int y = j0 + r;
            gv = y >= 0 && y < ny && gx >= 0 && gx < nx;
            // offset from the parity base, not fo[c]: a per-lane index into fo[]
            // would put the pointer array in scratch and make every load generic
            gp = G(p.fbase[par]) + (size_t)c * p.fstride + (size_t)min(max(y, 0), ny - 1) * p.pitch +
                 min(max(gx, 0), nx - 1);
        }
        const size_t plane_elems = (size_t)ny * p.pitch;
        auto gather = [&](int kk) -> float {
            const float v = gp[(size_t)kk * plane_elems];
            return gv ? v : 0.f;
        };

        float hcx[TY + 1], hcy[TY + 1], hcz[TY];   // H_old(k) rows 0..TY (z = k)
        float ecx[TY + 1], ecy[TY], ecz[TY + 1];    // E_new(k)
        float hxr_m[TY], hyr_m[TY];                 // H_x, H_y at x0+64, plane k (uniform)
        float eyr[TY], ezr[TY];                     // E_new(k) at x0+64 (uniform)
        double en = 0.0;

        // E_new on plane kk from H_old(kk) (h*) and H_old(kk-1) (hm*); e* hold
        // E_old on entry. Row TY is formed for the H update of row TY-1.
        auto e_new = [&](int kk, const float (&hx)[TY + 2], const float (&hy)[TY + 1],
                         const float (&hz)[TY + 2], const float (&hmx)[TY + 1],
                         const float (&hmy)[TY + 1], float g, float (&ex)[TY + 1],
                         float (&ey)[TY + 1], float (&ez)[TY + 1]) {
            float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
            if (p.colmap) {
                const float2 tt = ldc2(p.tE, n);
                pt0 = cmul(ldc2(p.zph, 2 * kk), tt);
                pt1 = cmul(ldc2(p.zph, 2 * kk + 1), tt);
            }
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                float hy_im = __shfl_up(hy[r], 1, 64);
                float hz_im = __shfl_up(hz[r + 1], 1, 64);
                if (lane == 0) {
                    hy_im = hl ? bcastb(g, H::L_HY + r) : 0.f;
                    hz_im = hl ? bcastb(g, H::L_HZ + r) : 0.f;
                }
                if (!xin || !rv[r + 1]) {
                    ex[r] = ey[r] = ez[r] = 0.f;
                    continue;
                }
                HNbr h;
                h.hx = hx[r + 1];
                h.hx_jm = hx[r];
                h.hx_km = hmx[r];
                h.hy = hy[r];
                h.hy_im = hy_im;
                h.hy_km = hmy[r];
                h.hz = hz[r + 1];
                h.hz_im = hz_im;
                h.hz_jm = hz[r];
                e_cell<true>(p, par, x, j0 + r, kk, h, ex[r], ey[r], ez[r], slot[r], pt0, pt1,
                             r < TY && owned(r));
            }
        };
        // E_new(E_y, E_z) at x0+64, rows 0..TY-1, wavefront-uniform; lane 63's
        // H at x0+63 comes in by readlane. Updates the carried H at x0+64.
        auto e_right = [&](int kk, const float (&hy)[TY + 1], const float (&hz)[TY + 2], float g) {
            float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
            if (p.colmap) {
                const float2 tt = ldc2(p.tE, n);
                pt0 = cmul(ldc2(p.zph, 2 * kk), tt);
                pt1 = cmul(ldc2(p.zph, 2 * kk + 1), tt);
            }
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const float hxv = bcastb(g, H::R_HX + 1 + r), hyv = bcastb(g, H::R_HY + r);
                if (!hr || j0 + r >= ny) {
                    eyr[r] = ezr[r] = 0.f;
                } else {
                    HNbr h;
                    h.hx = hxv;
                    h.hx_jm = bcastb(g, H::R_HX + r);
                    h.hx_km = hxr_m[r];
                    h.hy = hyv;
                    h.hy_im = bcastb(hy[r], 63);
                    h.hy_km = hyr_m[r];
                    h.hz = bcastb(g, H::R_HZ + 1 + r);
                    h.hz_im = bcastb(hz[r + 1], 63);
                    h.hz_jm = bcastb(g, H::R_HZ + r);
                    float vx = bcastb(g, H::R_EX + r), vy = bcastb(g, H::R_EY + r),
                          vz = bcastb(g, H::R_EZ + r);
                    e_cell<true>(p, par, x0 + SEG, j0 + r, kk, h, vx, vy, vz, slot_h[r], pt0, pt1,
                                 false);
                    eyr[r] = vy;
                    ezr[r] = vz;
                }
                hxr_m[r] = hxv;
                hyr_m[r] = hyv;
            }
        };
        auto store_e = [&](int kk, const float (&ex)[TY + 1], const float (&ey)[TY + 1],
                           const float (&ez)[TY + 1]) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (!owned(r)) continue;
                const size_t pk = (size_t)kk * plane;
                stb(fw[EX] + pk, ro[r + 1], ex[r]);
                stb(fw[EY] + pk, ro[r + 1], ey[r]);
                stb(fw[EZ] + pk, ro[r + 1], ez[r]);
                if (epart) en += (double)ex[r] * ex[r] + (double)ey[r] * ey[r] + (double)ez[r] * ez[r];
                if (kk == p.plane) {
                    const size_t pl = (size_t)(j0 + r) * nx + x, ps = (size_t)nx * ny;
                    const gptr<double> fl = G(p.fl);
                    if (mask & FDTD_DIAG_EX2) fl[pl] = sq_acc(fl[pl], ex[r]);
                    if (mask & FDTD_DIAG_EY2) fl[ps + pl] = sq_acc(fl[ps + pl], ey[r]);
                    if (mask & FDTD_DIAG_EZ2) fl[2 * ps + pl] = sq_acc(fl[2 * ps + pl], ez[r]);
                    if (p.rec) G(p.rec)[(size_t)(n - p.rec_begin) * ps + pl] = ey[r];
                }
            }
        };

        // ---- prologue: E_new(kb) ----------------------------------------
        {
            const int km = kb == 0 ? nz - 1 : kb - 1;
            float hx[TY + 2], hy[TY + 1], hz[TY + 2], hmx[TY + 1], hmy[TY + 1];
            float ex[TY + 1], ey[TY + 1], ez[TY + 1];
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                hx[r + 1] = ld(HX, kb, r);
                hz[r + 1] = ld(HZ, kb, r);
                if (r >= 0) {
                    hy[r] = ld(HY, kb, r);
                    hmx[r] = ld(HX, km, r);
                    hmy[r] = ld(HY, km, r);
                    ex[r] = ld(EX, kb, r);
                    ey[r] = ld(EY, kb, r);
                    ez[r] = ld(EZ, kb, r);
                }
            }
            const float gm = gather(km), g0 = gather(kb);
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                hxr_m[r] = bcastb(gm, H::R_HX + 1 + r);
                hyr_m[r] = bcastb(gm, H::R_HY + r);
            }
            e_new(kb, hx, hy, hz, hmx, hmy, g0, ex, ey, ez);
            e_right(kb, hy, hz, g0);
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                hcx[r] = hx[r + 1];
                hcy[r] = hy[r];
                ecx[r] = ex[r];
                ecz[r] = ez[r];
                if (r < TY) {
                    hcz[r] = hz[r + 1];
                    ecy[r] = ey[r];
                }
            }
            store_e(kb, ex, ey, ez);
        }
        const float2 th = p.colmap ? ldc2(p.tH, n) : make_float2(0.f, 0.f);

        for (int k = kb; k < ke; ++k) {
            const int kn = k + 1 == nz ? 0 : k + 1;
            float hx[TY + 2], hy[TY + 1], hz[TY + 2];
            float ex[TY + 1], ey[TY + 1], ez[TY + 1];
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                hx[r + 1] = ld(HX, kn, r);
                hz[r + 1] = ld(HZ, kn, r);
                if (r >= 0) {
                    hy[r] = ld(HY, kn, r);
                    ex[r] = ld(EX, kn, r);
                    ey[r] = ld(EY, kn, r);
                    ez[r] = ld(EZ, kn, r);
                }
            }
            const float gn = gather(kn);
            // ---- H_new(k) needs E_new(k) at x0+64 and E_new(k+1) ----------
            float eyr_k[TY], ezr_k[TY];
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                eyr_k[r] = eyr[r];
                ezr_k[r] = ezr[r];
            }
            e_new(kn, hx, hy, hz, hcx, hcy, gn, ex, ey, ez);
            e_right(kn, hy, hz, gn);
            float2 qt0 = make_float2(0.f, 0.f), qt1 = qt0;
            if (p.colmap) {
                qt0 = cmul(ldc2(p.zph, 2 * k), th);
                qt1 = cmul(ldc2(p.zph, 2 * k + 1), th);
            }
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (!owned(r)) continue;
                float ey_ip = __shfl_down(ecy[r], 1, 64);
                float ez_ip = __shfl_down(ecz[r], 1, 64);
                if (lane == 63) {
                    ey_ip = eyr_k[r];
                    ez_ip = ezr_k[r];
                }
                ENbr e;
                e.ex = ecx[r];
                e.ex_jp = ecx[r + 1];
                e.ex_kp = ex[r];
                e.ey = ecy[r];
                e.ey_ip = ey_ip;
                e.ey_kp = ey[r];
                e.ez = ecz[r];
                e.ez_ip = ez_ip;
                e.ez_jp = ecz[r + 1];
                float vx = hcx[r], vy = hcy[r], vz = hcz[r];
                h_cell<true>(p, par, x, j0 + r, k, e, vx, vy, vz, slot[r], qt0, qt1);
                const size_t pk = (size_t)k * plane;
                stb(fw[HX] + pk, ro[r + 1], vx);
                stb(fw[HY] + pk, ro[r + 1], vy);
                stb(fw[HZ] + pk, ro[r + 1], vz);
                if (epart) en += (double)hcx[r] * vx + (double)hcy[r] * vy + (double)hcz[r] * vz;
            }
            if (k + 1 < ke) store_e(kn, ex, ey, ez);
            // ---- rotate -------------------------------------------------------
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                hcx[r] = hx[r + 1];
                hcy[r] = hy[r];
                ecx[r] = ex[r];
                ecz[r] = ez[r];
                if (r < TY) {
                    hcz[r] = hz[r + 1];
                    ecy[r] = ey[r];
                }
            }
        }
        if (epart) {
            en = wave_sum(en);
            if (lane == 0) epart[t] = en;
        }
    }
}

}  // namespace

hipError_t launch_fused_bnd(const Problem& single, const Problem* probs, const int4* tiles,
                            int ntiles, int rows, int cz, int blocks, const long long* nctr,
                            long long n_off, int par, int diag, const Frame& excl, double* epart,
                            hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (rows != 2 && rows != 4) return hipErrorInvalidValue;
    const dim3 g(blocks), b(64 * WAVES);
    if (probs && rows == 4)
        hipLaunchKernelGGL((fused_bnd_kernel<4, true>), g, b, 0, s, single, probs, tiles, ntiles,
                           cz, nctr, n_off, par, diag, excl, epart);
    else if (probs)
        hipLaunchKernelGGL((fused_bnd_kernel<2, true>), g, b, 0, s, single, probs, tiles, ntiles,
                           cz, nctr, n_off, par, diag, excl, epart);
    else if (rows == 4)
        hipLaunchKernelGGL((fused_bnd_kernel<4, false>), g, b, 0, s, single, probs, tiles, ntiles,
                           cz, nctr, n_off, par, diag, excl, epart);
    else
        hipLaunchKernelGGL((fused_bnd_kernel<2, false>), g, b, 0, s, single, probs, tiles, ntiles,
                           cz, nctr, n_off, par, diag, excl, epart);
    return hipGetLastError();
}

int fused_bnd_blocks_per_cu(int rows, bool multi) {
    int b = 0;
    hipError_t e;
    if (rows == 4)
        e = multi ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fused_bnd_kernel<4, true>,
                                                                 64 * WAVES, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fused_bnd_kernel<4, false>,
                                                                 64 * WAVES, 0);
    else
        e = multi ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fused_bnd_kernel<2, true>,
                                                                 64 * WAVES, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fused_bnd_kernel<2, false>,
                                                                 64 * WAVES, 0);
    if (e != hipSuccess) return 1;
    return b > 0 ? b : 1;
}

}  // namespace bfdtd
