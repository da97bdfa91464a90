// Fused Yee step on the interior of the grid: E update + E source, then
// H update + H source, in one kernel that reads the old ping-pong buffers
// once and writes the new ones once (48 B of field traffic per cell-update).
// The interior is the rectangle of cells whose stencils touch no wall, no
// CPML slab and no periodic wrap in x/y; the frame around it runs through
// the split kernels (kernels_split.hip), which carry every boundary case.
//
// Work decomposition (CDNA4, wave64). A wavefront owns a block of 64 x cells
// (a 256-byte row segment starting on a 128-byte line, so every load and
// store covers whole lines) × TY y rows and marches along z over a chunk of
// planes, keeping two planes of each field in registers.
//   * x: lane l holds x = x0 + l; x neighbours move between lanes with
//     cross-lane shuffles. The halo columns x0-1 (H for lane 0) and x0+64
//     (from which E_new at x0+64 is formed for lane 63) are fetched per plane
//     by one gather instruction, one value per lane, and broadcast to the
//     wavefront with readlane; the x0+64 update is done wavefront-uniform.
//     Wavefronts never wait for each other: there is no barrier, so each
//     keeps its own loads in flight.
//   * y: each lane holds rows j0-1 .. j0+TY of H and j0 .. j0+TY of E in
//     registers; E_new of row j0+TY is recomputed for the H update of the
//     last owned row. A workgroup stacks four wavefronts of the same x
//     segment in y, so the halo rows they share are fetched by one CU at
//     about the same time.
//   * z: E_new(k+1) is formed from H_old(k+1) and H_old(k), then H_new(k)
//     from E_new(k) and E_new(k+1); the z index wraps (periodic axis).
// Addresses are a uniform component base (scalar registers) plus a 32-bit
// per-lane byte offset; components of 4 GiB or more use a 64-bit plane base
// instead, with the 32-bit offset inside the plane. The new fields are written with non-temporal stores:
// nothing reads them again in this launch, and keeping them out of the
// caches leaves room for the halo rows that neighbouring tiles re-read.
// Hardware block b runs on XCD b % 8; the block index is remapped so each
// XCD receives a contiguous run of tiles and the y-halo rows shared by
// neighbouring tiles stay in one L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int WAVES = 4;   // wavefronts per workgroup, stacked in y
constexpr int SEG = 64;    // x cells per wavefront

__device__ __forceinline__ float ldo(const float* base, unsigned boff) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + boff);
}

__device__ __forceinline__ void sto(float* base, unsigned boff, float v) {
    __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + boff));
}

// Interior geometry: segment s covers x in [x_org + 64 s, x_org + 64 s + 64),
// row group g covers y in [y_org + TY g, y_org + TY g + TY).
struct Interior {
    int x_org, y_org, nseg, nrow, ncz, cz;
};

// BIG: a field component spans 4 GiB or more, so plane bases are 64-bit
// (scalar) and only the in-plane offset is 32-bit; otherwise the whole
// offset is one 32-bit value.
template <int TY, bool BIG>
struct Tile {
    const Problem& p;
    int x, j0, lane;
    unsigned ro[TY + 2];   // byte offset of (row j0 + r, x) in a plane, r = -1..TY
    size_t plane;          // floats per plane
    unsigned pstride;      // bytes per plane (when !BIG)
    const float* fo[6];    // component bases, old parity
    float* fw[6];          // component bases, new parity

    __device__ Tile(const Problem& pp, int par, int x0, int jj0) : p(pp), j0(jj0) {
        lane = threadIdx.x & 63;
        x = x0 + lane;
#pragma unroll
        for (int r = -1; r <= TY; ++r) ro[r + 1] = 4u * (unsigned)((j0 + r) * p.pitch + x);
        plane = (size_t)p.ny * p.pitch;
        pstride = 4u * (unsigned)plane;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            fo[c] = p.fbase[par] + c * p.fstride;
            fw[c] = p.fbase[par ^ 1] + c * p.fstride;
        }
    }
    __device__ float ld(int c, int kk, int r) const {
        if (BIG) return ldo(fo[c] + (size_t)kk * plane, ro[r + 1]);
        return ldo(fo[c], (unsigned)kk * pstride + ro[r + 1]);
    }
    __device__ void st(int c, int kk, int r, float v) const {
        if (BIG)
            sto(fw[c] + (size_t)kk * plane, ro[r + 1], v);
        else
            sto(fw[c], (unsigned)kk * pstride + ro[r + 1], v);
    }
};

// E_new on plane kk, rows 0..TY (ex/ey/ez hold E_old on entry); hx/hy/hz are
// H_old(kk) (rows -1..TY, 0..TY, -1..TY), hxm/hym H_old(kk-1); hyl/hzl: H at
// x0-1 for lane 0.
template <int TY>
__device__ __forceinline__ void e_plane(const Problem& p, int lane, long long n, int kk,
                                        const int (&slot)[TY + 1], const float (&hx)[TY + 2],
                                        const float (&hy)[TY + 1], const float (&hz)[TY + 2],
                                        const float (&hxm)[TY], const float (&hym)[TY + 1],
                                        const float (&hyl)[TY + 1], const float (&hzl)[TY],
                                        float (&ex)[TY + 1], float (&ey)[TY], float (&ez)[TY + 1]) {
    float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
    if (p.colmap) {
        const float2 t = ldc2(p.tE, n);
        pt0 = cmul(ldc2(p.zph, 2 * kk), t);
        pt1 = cmul(ldc2(p.zph, 2 * kk + 1), t);
    }
#pragma unroll
    for (int r = 0; r <= TY; ++r) {
        float hz_im = __shfl_up(hz[r + 1], 1, 64);
        float hy_im = __shfl_up(hy[r], 1, 64);
        if (lane == 0) {
            hy_im = hyl[r];
            if (r < TY) hz_im = hzl[r];
        }
        // E_x += S_y Δ_y H_z - S_z Δ_z H_y
        ex[r] += curl_pair(p.sy, hz[r + 1] - hz[r], p.sz, hy[r] - hym[r]);
        // E_z += S_x Δ_x H_y - S_y Δ_y H_x
        ez[r] += curl_pair(p.sx, hy[r] - hy_im, p.sy, hx[r + 1] - hx[r]);
        // E_y += S_z Δ_z H_x - S_x Δ_x H_z
        if (r < TY) ey[r] += curl_pair(p.sz, hx[r + 1] - hxm[r < TY ? r : 0], p.sx, hz[r + 1] - hz_im);
        if (slot[r] >= 0) {
            const float2* a = p.amp + (size_t)slot[r] * 6;
            ex[r] += cmul_re(a[EX], pt0);
            ez[r] += cmul_re(a[EZ], pt1);
            if (r < TY) ey[r] += cmul_re(a[EY], pt0);
        }
    }
}

// Halo columns. Lane 0 needs H_y (rows 0..TY) and H_z (rows 0..TY-1) at
// x0-1; lane 63 needs E_new(E_y, E_z) at x0+64 (rows 0..TY-1), formed from
// H_x (rows -1..TY-1), H_y, H_z, E_y, E_z (rows 0..TY-1) of that column.
// Those 7 TY + 2 values of one plane are fetched by a single gather: lane q
// loads value q, and the wavefront broadcasts them with readlane.
template <int TY>
struct Halo {
    static constexpr int R_HX = 0;              // x0+64: H_x rows -1..TY-1
    static constexpr int R_HY = TY + 1;         //        H_y rows 0..TY-1
    static constexpr int R_HZ = 2 * TY + 1;     //        H_z
    static constexpr int R_EY = 3 * TY + 1;     //        E_y
    static constexpr int R_EZ = 4 * TY + 1;     //        E_z
    static constexpr int L_HY = 5 * TY + 1;     // x0-1:  H_y rows 0..TY
    static constexpr int L_HZ = 6 * TY + 2;     //        H_z rows 0..TY-1
    static constexpr int COUNT = 7 * TY + 2;
    static_assert(COUNT <= 64, "halo gather exceeds one wavefront");
};

__device__ __forceinline__ float bcast(float v, int q) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), q));
}

// Element offset (from the old-parity field base, plane 0) of halo value q.
template <int TY>
__device__ __forceinline__ size_t halo_offset(const Problem& p, int q, int j0, int x0) {
    using Hq = Halo<TY>;
    int c = HX, r = -1, x = x0 + SEG;
    if (q >= Hq::L_HZ) { c = HZ; r = q - Hq::L_HZ; x = x0 - 1; }
    else if (q >= Hq::L_HY) { c = HY; r = q - Hq::L_HY; x = x0 - 1; }
    else if (q >= Hq::R_EZ) { c = EZ; r = q - Hq::R_EZ; }
    else if (q >= Hq::R_EY) { c = EY; r = q - Hq::R_EY; }
    else if (q >= Hq::R_HZ) { c = HZ; r = q - Hq::R_HZ; }
    else if (q >= Hq::R_HY) { c = HY; r = q - Hq::R_HY; }
    else { r = q - 1; }
    return (size_t)c * p.fstride + (size_t)(j0 + r) * p.pitch + x;
}

// E_new(E_y, E_z) at x0+64, rows 0..TY-1, of plane kk from the gathered
// column g (uniform) and H at x0+63 (lane 63's registers; other lanes form
// values nobody reads). hxkm: H_x(x0+64) of plane kk-1, replaced by plane kk.
template <int TY>
__device__ __forceinline__ void e_halo_right(const Problem& p, long long n, int kk, float g,
                                             const int (&slot_h)[TY],
                                             const float (&hy)[TY + 1], const float (&hz)[TY + 2],
                                             float (&hxkm)[TY], float (&ey_h)[TY],
                                             float (&ez_h)[TY]) {
    using Hq = Halo<TY>;
    float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
    if (p.colmap) {
        const float2 t = ldc2(p.tE, n);
        pt0 = cmul(ldc2(p.zph, 2 * kk), t);
        pt1 = cmul(ldc2(p.zph, 2 * kk + 1), t);
    }
    float hx_prev = bcast(g, Hq::R_HX);
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        const float hxr = bcast(g, Hq::R_HX + 1 + r);
        // same association as e_plane (E + (curl)), so the column matches the
        // value its own segment forms bit for bit
        float vy = bcast(g, Hq::R_EY + r);
        vy += curl_pair(p.sz, hxr - hxkm[r], p.sx, bcast(g, Hq::R_HZ + r) - hz[r + 1]);
        float vz = bcast(g, Hq::R_EZ + r);
        vz += curl_pair(p.sx, bcast(g, Hq::R_HY + r) - hy[r], p.sy, hxr - hx_prev);
        if (slot_h[r] >= 0) {
            const float2* a = p.amp + (size_t)slot_h[r] * 6;
            vy += cmul_re(a[EY], pt0);
            vz += cmul_re(a[EZ], pt1);
        }
        ey_h[r] = vy;
        ez_h[r] = vz;
        hxkm[r] = hxr;
        hx_prev = hxr;
    }
}

template <int TY, bool BIG>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(TY == 4 ? 3 : 2)))
fused_interior_kernel(Problem p, long long n, int par, Interior I, int nblocks_padded,
                      double* epart) {
    // ---- which tile: hardware block b runs on XCD b % 8 ----------------
    const int nrq = (I.nrow + WAVES - 1) / WAVES;              // row groups per workgroup
    const int lb = (blockIdx.x % 8) * (nblocks_padded / 8) + blockIdx.x / 8;
    if (lb >= I.nseg * nrq * I.ncz) return;                    // whole workgroup
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int seg = lb % I.nseg;
    const int sy = ((lb / I.nseg) % nrq) * WAVES + w;
    const int kb = (lb / (I.nseg * nrq)) * I.cz;
    const int ke = min(kb + I.cz, p.nz);
    double* epart_slot = epart ? epart + ((size_t)lb * WAVES + w) : nullptr;
    if (sy >= I.nrow) {                                        // uniform per wavefront
        if (epart_slot && (threadIdx.x & 63) == 0) *epart_slot = 0.0;
        return;
    }
    const int j0 = I.y_org + sy * TY;
    const Tile<TY, BIG> T(p, par, I.x_org + SEG * seg, j0);
    const int lane = T.lane;
    const int nz = p.nz, nx = p.nx, ny = p.ny;
    const bool right = lane == 63;

    const int x0 = I.x_org + SEG * seg;
    int slot[TY + 1], slot_h[TY];
#pragma unroll
    for (int r = 0; r <= TY; ++r) slot[r] = p.colmap ? p.colmap[(size_t)(j0 + r) * nx + T.x] : -1;
#pragma unroll
    for (int r = 0; r < TY; ++r)
        slot_h[r] = p.colmap ? p.colmap[(size_t)(j0 + r) * nx + x0 + SEG] : -1;
    // halo gather: lane q < Halo::COUNT fetches halo value q of each plane
    const float* gbase = p.fbase[par] +
                         halo_offset<TY>(p, lane < Halo<TY>::COUNT ? lane : 0, j0, x0);
    const size_t plane_elems = (size_t)ny * p.pitch;
    auto gather = [&](int kk) { return gbase[(size_t)kk * plane_elems]; };

    float hcx[TY], hcy[TY + 1], hcz[TY];      // H_old(k), kept for the H update
    float ecx[TY + 1], ecy[TY], ecz[TY + 1];  // E_new(k)
    float hxh[TY], eyh[TY], ezh[TY];          // H_x(k), E_new(k) at x0+64 (uniform)
    float hyl[TY + 1], hzl[TY];               // H at x0-1 (uniform)

    auto get_left = [&](float g) {
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            hyl[r] = bcast(g, Halo<TY>::L_HY + r);
            if (r < TY) hzl[r] = bcast(g, Halo<TY>::L_HZ + r);
        }
    };

    double en = 0.0;
    auto store_e = [&](int kk, const float (&ex)[TY + 1], const float (&ey)[TY],
                       const float (&ez)[TY + 1]) {
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            T.st(EX, kk, r, ex[r]);
            T.st(EY, kk, r, ey[r]);
            T.st(EZ, kk, r, ez[r]);
            if (epart_slot) en += (double)ex[r] * ex[r] + (double)ey[r] * ey[r] + (double)ez[r] * ez[r];
            if (kk == p.plane) {
                const size_t pl = (size_t)(j0 + r) * nx + T.x, ps = (size_t)nx * ny;
                if (p.diag_mask & FDTD_DIAG_EX2) p.fl[pl] = sq_acc(p.fl[pl], ex[r]);
                if (p.diag_mask & FDTD_DIAG_EY2) p.fl[ps + pl] = sq_acc(p.fl[ps + pl], ey[r]);
                if (p.diag_mask & FDTD_DIAG_EZ2) p.fl[2 * ps + pl] = sq_acc(p.fl[2 * ps + pl], ez[r]);
                if (p.rec) p.rec[(size_t)(n - p.rec_begin) * ps + pl] = ey[r];
            }
        }
    };

    // ---- prologue: E_new(kb) ------------------------------------------
    {
        const int km = kb == 0 ? nz - 1 : kb - 1;
        float hx[TY + 2], hy[TY + 1], hz[TY + 2], hxm[TY], hym[TY + 1];
#pragma unroll
        for (int r = -1; r <= TY; ++r) {
            hx[r + 1] = T.ld(HX, kb, r);
            hz[r + 1] = T.ld(HZ, kb, r);
            if (r >= 0) {
                hy[r] = T.ld(HY, kb, r);
                hym[r] = T.ld(HY, km, r);
                ecx[r] = T.ld(EX, kb, r);
                ecz[r] = T.ld(EZ, kb, r);
            }
            if (r >= 0 && r < TY) {
                hxm[r] = T.ld(HX, km, r);
                ecy[r] = T.ld(EY, kb, r);
            }
        }
        const float gm = gather(km), g0 = gather(kb);
        get_left(g0);
        e_plane<TY>(p, lane, n, kb, slot, hx, hy, hz, hxm, hym, hyl, hzl, ecx, ecy, ecz);
#pragma unroll
        for (int r = 0; r < TY; ++r) hxh[r] = bcast(gm, Halo<TY>::R_HX + 1 + r);
        e_halo_right<TY>(p, n, kb, g0, slot_h, hy, hz, hxh, eyh, ezh);
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            hcx[r] = hx[r + 1];
            hcy[r] = hy[r];
            hcz[r] = hz[r + 1];
        }
        hcy[TY] = hy[TY];
        store_e(kb, ecx, ecy, ecz);
    }
    const float2 th = p.colmap ? ldc2(p.tH, n) : make_float2(0.f, 0.f);

    for (int k = kb; k < ke; ++k) {
        const int kn = k + 1 == nz ? 0 : k + 1;
        float hx[TY + 2], hy[TY + 1], hz[TY + 2];
        float enx[TY + 1], eny[TY], enz[TY + 1];
#pragma unroll
        for (int r = -1; r <= TY; ++r) {
            hx[r + 1] = T.ld(HX, kn, r);
            hz[r + 1] = T.ld(HZ, kn, r);
            if (r >= 0) {
                hy[r] = T.ld(HY, kn, r);
                enx[r] = T.ld(EX, kn, r);
                enz[r] = T.ld(EZ, kn, r);
            }
            if (r >= 0 && r < TY) eny[r] = T.ld(EY, kn, r);
        }
        const float gn = gather(kn);
        // ---- E_new(k+1) -------------------------------------------------
        get_left(gn);
        e_plane<TY>(p, lane, n, kn, slot, hx, hy, hz, hcx, hcy, hyl, hzl, enx, eny, enz);
        float eyh_n[TY], ezh_n[TY];
        e_halo_right<TY>(p, n, kn, gn, slot_h, hy, hz, hxh, eyh_n, ezh_n);

        // ---- H_new(k) ---------------------------------------------------
        float2 qt0 = make_float2(0.f, 0.f), qt1 = qt0;
        if (p.colmap) {
            qt0 = cmul(ldc2(p.zph, 2 * k), th);
            qt1 = cmul(ldc2(p.zph, 2 * k + 1), th);
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            float ey_ip = __shfl_down(ecy[r], 1, 64);
            float ez_ip = __shfl_down(ecz[r], 1, 64);
            if (right) {
                ey_ip = eyh[r];
                ez_ip = ezh[r];
            }
            // H_x -= S_y Δ_y E_z - S_z Δ_z E_y
            float vx = hcx[r] - (curl_pair(p.sy, ecz[r + 1] - ecz[r], p.sz, eny[r] - ecy[r]));
            // H_y -= S_z Δ_z E_x - S_x Δ_x E_z
            float vy = hcy[r] - (curl_pair(p.sz, enx[r] - ecx[r], p.sx, ez_ip - ecz[r]));
            // H_z -= S_x Δ_x E_y - S_y Δ_y E_x
            float vz = hcz[r] - (curl_pair(p.sx, ey_ip - ecy[r], p.sy, ecx[r + 1] - ecx[r]));
            if (slot[r] >= 0) {
                const float2* a = p.amp + (size_t)slot[r] * 6;
                vx += cmul_re(a[HX], qt1);
                vy += cmul_re(a[HY], qt1);
                vz += cmul_re(a[HZ], qt0);
            }
            T.st(HX, k, r, vx);
            T.st(HY, k, r, vy);
            T.st(HZ, k, r, vz);
            if (epart_slot) en += (double)hcx[r] * vx + (double)hcy[r] * vy + (double)hcz[r] * vz;
        }
        if (k + 1 < ke) store_e(kn, enx, eny, enz);
        // ---- rotate -----------------------------------------------------
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            hcx[r] = hx[r + 1];
            hcy[r] = hy[r];
            hcz[r] = hz[r + 1];
            ecy[r] = eny[r];
        }
        hcy[TY] = hy[TY];
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            ecx[r] = enx[r];
            ecz[r] = enz[r];
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            eyh[r] = eyh_n[r];
            ezh[r] = ezh_n[r];
        }
    }
    if (epart_slot) {
        en = wave_sum(en);
        if (lane == 0) *epart_slot = en;
    }
}

// Interior: x0 - 1 >= m and every x0 a multiple of xalign floats (32: a
// 128-byte line; 64: whole 64-cell tiles of the frame kernel to the left);
// the last segment keeps its column x0 + 64 inside too; rows j0 - 1 ..
// j0 + TY likewise, m = max(npml, 1), upper bound n - npml - 1.
Interior interior(const Problem& p, int rows, int zchunk, int xalign) {
    Interior I{0, 0, 0, 0, 0, 0};
    if (p.periodic) return I;
    const int m = p.npml > 0 ? p.npml : 1;
    const int hi_x = p.nx - p.npml - 1, hi_y = p.ny - p.npml - 1;
    I.x_org = (m + 1 + xalign - 1) / xalign * xalign;
    I.y_org = m + 1;
    I.nseg = hi_x - I.x_org - SEG + 1 >= 0 ? (hi_x - I.x_org - SEG) / SEG + 1 : 0;
    I.nrow = hi_y - I.y_org - rows + 1 >= 0 ? (hi_y - I.y_org - rows) / rows + 1 : 0;
    I.cz = zchunk > 0 ? min(zchunk, p.nz) : p.nz;
    I.ncz = (p.nz + I.cz - 1) / I.cz;
    if (I.nseg <= 0 || I.nrow <= 0) I.nseg = I.nrow = 0;
    return I;
}

int group_count(const Interior& I) {
    return I.nseg * ((I.nrow + WAVES - 1) / WAVES) * I.ncz;
}

template <int TY>
hipError_t launch_rows(const Problem& p, long long n, int parity, int zchunk, int xalign,
                       double* epart, hipStream_t s, LaunchTimer* timer) {
    const Interior I = interior(p, TY, zchunk, xalign);
    const int nb = group_count(I);
    if (nb <= 0) return hipSuccess;
    const int nbp = (nb + 7) / 8 * 8;
    if (timer) timer->mark("fused_interior");
    if ((size_t)p.fstride * sizeof(float) >= ((size_t)1 << 32))
        hipLaunchKernelGGL((fused_interior_kernel<TY, true>), dim3(nbp), dim3(64 * WAVES), 0, s,
                           p, n, parity, I, nbp, epart);
    else
        hipLaunchKernelGGL((fused_interior_kernel<TY, false>), dim3(nbp), dim3(64 * WAVES), 0, s,
                           p, n, parity, I, nbp, epart);
    return hipGetLastError();
}

}  // namespace

Frame fused_interior_rect(const Problem& p, int rows, int xalign) {
    const Interior I = interior(p, rows, 0, xalign);
    if (I.nseg <= 0) return Frame{0, 0, 0, 0};
    return Frame{I.x_org, I.x_org + SEG * I.nseg, I.y_org, I.y_org + rows * I.nrow};
}

int fused_default_zchunk(const Problem& p, int rows, int xalign, int cus) {
    const Interior I = interior(p, rows, 0, xalign);
    if (I.nseg <= 0) return 0;
    const long long base = group_count(I);          // workgroups with the whole z
    const long long target = 32LL * (cus > 0 ? cus : 256);
    if (base >= target) return 0;
    const long long chunks = (target + base - 1) / base;
    const int cz = (int)std::max<long long>(4, (p.nz + chunks - 1) / chunks);
    return cz >= p.nz ? 0 : cz;
}

int fused_interior_tiles(const Problem& p, int rows, int zchunk, int xalign) {
    return group_count(interior(p, rows, zchunk, xalign)) * WAVES;
}

hipError_t launch_fused_interior(const Problem& p, long long n, int parity, int rows, int zchunk,
                                 int xalign, double* epart, hipStream_t s, LaunchTimer* timer) {
    if (xalign != 32 && xalign != 64) return hipErrorInvalidValue;
    if (rows == 4) return launch_rows<4>(p, n, parity, zchunk, xalign, epart, s, timer);
    if (rows == 8) return launch_rows<8>(p, n, parity, zchunk, xalign, epart, s, timer);
    return hipErrorInvalidValue;
}

// Deterministic single-block sum of the energy partials.
__global__ void __launch_bounds__(256) energy_reduce_kernel(const double* part, int n, double* out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) v += part[q];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_energy_reduce(const double* part, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(energy_reduce_kernel, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

}  // namespace bfdtd
