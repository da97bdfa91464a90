// Fused Yee step: E update + E source, then H update + H source, in one
// kernel, reading the old ping-pong buffers once and writing the new ones
// once (48 B of field traffic per cell-update, plus CPML memories).
//
// Work decomposition (CDNA4, wave64). Every wavefront is independent (no LDS,
// no barriers): it owns a column block of 62 x cells × TY y rows and marches
// along z over a chunk of planes, keeping two planes of each field in
// registers.
//   * x: lane l sits at x = 62·seg - 1 + l. Lanes 1..62 own their cell;
//     lane 0 supplies H at x-1 to lane 1, lane 63 supplies E_new at x+1 to
//     lane 62 (it recomputes E there). x neighbours move between lanes with
//     cross-lane shuffles.
//   * y: each lane holds rows j0-1 .. j0+TY of H and j0 .. j0+TY of E in
//     registers; E_new of row j0+TY is recomputed for the H update of the
//     last owned row.
//   * z: E_new(k+1) is formed from H_old(k+1) and H_old(k), then H_new(k)
//     from E_new(k) and E_new(k+1); the z index wraps (periodic axis).
// Addresses are a uniform row pointer (scalar registers) plus one per-lane
// byte offset, so a load costs one vector register for its address.
// Wavefronts whose cells touch no wall, CPML slab or periodic wrap run a
// lean interior path; the others run the general path with all boundary
// logic. Consecutive workgroups are spread over the 8 XCDs by the hardware;
// the block index is remapped so each XCD receives a contiguous run of tiles
// and the y-halo rows shared by neighbouring tiles stay in one L2.
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"

namespace bfdtd {

namespace {

constexpr int WAVES_PER_BLOCK = 4;
constexpr int SEG = 62;   // owned x cells per wavefront

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Load / store at a 32-bit byte offset from a uniform row pointer.
__device__ __forceinline__ float ldo(const float* row, unsigned boff) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(row) + boff);
}

__device__ __forceinline__ void sto(float* row, unsigned boff, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(row) + boff) = v;
}

__device__ __forceinline__ float cpml_term(float d, float b, float c, float kinv, float& psi,
                                           bool update) {
    if (update) psi = b * psi + c * d;
    return kinv * d + psi;
}

// Per-wave geometry. For the interior path every flag is constant.
template <int TY, bool EDGE>
struct Geo {
    const Problem& p;
    int par;
    int x, xl;           // lane x, addressing x
    unsigned xo;         // byte offset of xl in a row
    bool xv, own_x, hold_x, zero_x;
    int xs;              // x-slab index (EDGE only)
    int j0;
    int jl[TY + 2];      // addressing row of r = -1..TY (index r+1)
    bool jv[TY + 2];
    int ys[TY + 2];
    unsigned ro[TY + 2]; // per-lane byte offset of (row r, x) inside a plane
    const float* fo[6];  // component bases, old parity
    float* fw[6];        // component bases, new parity
    unsigned pstride;    // bytes per plane

    __device__ Geo(const Problem& pp, int parity, int seg, int jj0) : p(pp), par(parity), j0(jj0) {
        const int lane = threadIdx.x & 63;
        x = SEG * seg - 1 + lane;
        own_x = lane >= 1 && lane <= SEG && x < p.nx;
        if (!EDGE) {
            xl = x;
            xv = true;
            hold_x = zero_x = false;
            xs = -1;
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                jl[r + 1] = j0 + r;
                jv[r + 1] = true;
                ys[r + 1] = -1;
            }
        } else {
            const bool per = p.periodic != 0;
            if (per) {
                xl = wrap_mod(x, p.nx);
                xv = true;
            } else {
                xv = x >= 0 && x < p.nx;
                xl = xv ? x : 0;
            }
            xs = (x >= 0 && x < p.nx) ? slab_index(x, p.nx, p.npml) : -1;
            hold_x = !per && x == 0;
            zero_x = !per && !xv;
#pragma unroll
            for (int r = -1; r <= TY; ++r) {
                const int j = j0 + r;
                if (per) {
                    jl[r + 1] = wrap_mod(j, p.ny);
                    jv[r + 1] = true;
                } else {
                    jv[r + 1] = j >= 0 && j < p.ny;
                    jl[r + 1] = jv[r + 1] ? j : 0;
                }
                ys[r + 1] = (j >= 0 && j < p.ny) ? slab_index(j, p.ny, p.npml) : -1;
            }
        }
        xo = 4u * (unsigned)xl;
#pragma unroll
        for (int r = -1; r <= TY; ++r) ro[r + 1] = 4u * (unsigned)(jl[r + 1] * p.pitch) + xo;
        pstride = 4u * (unsigned)(p.ny * p.pitch);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            fo[c] = p.fbase[par] + c * p.fstride;
            fw[c] = p.fbase[par ^ 1] + c * p.fstride;
        }
    }
    __device__ bool own_y(int r) const { return r >= 0 && r < TY && (!EDGE || j0 + r < p.ny); }
    __device__ bool hold_y(int r) const {
        return EDGE && !p.periodic && jv[r + 1] && jl[r + 1] == 0;
    }
    __device__ bool zero(int r) const { return EDGE && (zero_x || !jv[r + 1]); }
    __device__ bool valid(int r) const { return !EDGE || (xv && jv[r + 1]); }
    __device__ float ld(int c, int kk, int r) const {
        const float v = ldo(fo[c], (unsigned)kk * pstride + ro[r + 1]);
        return valid(r) ? v : 0.0f;
    }
    __device__ void st(int c, int kk, int r, float v) const {
        sto(fw[c], (unsigned)kk * pstride + ro[r + 1], v);
    }
};

// E_new on plane kk, rows 0..TY (arrays ex/ey/ez hold E_old on entry).
template <int TY, bool EDGE>
__device__ __forceinline__ void e_plane(const Geo<TY, EDGE>& G, long long n, int kk,
                                        const int (&slot)[TY + 1], const float (&hx)[TY + 2],
                                        const float (&hy)[TY + 1], const float (&hz)[TY + 2],
                                        const float (&hxm)[TY], const float (&hym)[TY + 1],
                                        float (&ex)[TY + 1], float (&ey)[TY], float (&ez)[TY + 1],
                                        bool store_psi) {
    const Problem& p = G.p;
    float xb = 0.f, xc = 0.f, xk = 1.f;
    if (EDGE && G.xs >= 0) {
        xb = cx_tab(p, T_EB)[G.xl];
        xc = cx_tab(p, T_EC)[G.xl];
        xk = cx_tab(p, T_EK)[G.xl];
    }
    float2 pt0 = make_float2(0.f, 0.f), pt1 = pt0;
    if (p.colmap) {
        const float2 t = p.tE[n];
        pt0 = cmul(p.zph[2 * kk], t);
        pt1 = cmul(p.zph[2 * kk + 1], t);
    }
#pragma unroll
    for (int r = 0; r <= TY; ++r) {
        const float hz_im = __shfl_up(hz[r + 1], 1, 64);
        const float hy_im = __shfl_up(hy[r], 1, 64);
        float tyz = hz[r + 1] - hz[r];           // E_x: + S_y Δ_y H_z
        const float dzhy = hy[r] - hym[r];       //      - S_z Δ_z H_y
        float txy = hy[r] - hy_im;               // E_z: + S_x Δ_x H_y
        float tyx = hx[r + 1] - hx[r];           //      - S_y Δ_y H_x
        float txz = hz[r + 1] - hz_im;           // E_y: - S_x Δ_x H_z
        const float dzhx = r < TY ? hx[r + 1] - hxm[r < TY ? r : 0] : 0.f;   //  + S_z Δ_z H_x
        bool hy0 = false;
        if (EDGE) {
            hy0 = G.hold_y(r);
            const bool keep = store_psi && G.own_x && G.own_y(r);
            const int ys = G.ys[r + 1];
            if (ys >= 0) {
                const int jr = G.jl[r + 1];
                const float b = cy_tab(p, T_EB)[jr], c = cy_tab(p, T_EC)[jr];
                const float kinv = cy_tab(p, T_EK)[jr];
                const size_t q = psiy_at(p, kk, ys, G.xl);
                float px = pptr(p, G.par, P_EXY)[q], pz = pptr(p, G.par, P_EZY)[q];
                tyz = cpml_term(tyz, b, c, kinv, px, !hy0);
                tyx = cpml_term(tyx, b, c, kinv, pz, !hy0 && !G.hold_x);
                if (keep) {
                    pptr(p, G.par ^ 1, P_EXY)[q] = px;
                    pptr(p, G.par ^ 1, P_EZY)[q] = pz;
                }
            }
            if (G.xs >= 0) {
                const size_t q = psix_at(p, kk, G.jl[r + 1], G.xs);
                float pz = pptr(p, G.par, P_EZX)[q];
                txy = cpml_term(txy, xb, xc, xk, pz, !G.hold_x && !hy0);
                if (keep) pptr(p, G.par ^ 1, P_EZX)[q] = pz;
                if (r < TY) {
                    float py = pptr(p, G.par, P_EYX)[q];
                    txz = cpml_term(txz, xb, xc, xk, py, !G.hold_x);
                    if (keep) pptr(p, G.par ^ 1, P_EYX)[q] = py;
                }
            }
        }
        float vx = ex[r], vz = ez[r];
        if (!hy0) vx += p.sy * tyz - p.sz * dzhy;
        if (!hy0 && !(EDGE && G.hold_x)) vz += p.sx * txy - p.sy * tyx;
        float vy = 0.f;
        if (r < TY) {
            vy = ey[r];
            if (!(EDGE && G.hold_x)) vy += p.sz * dzhx - p.sx * txz;
        }
        if (slot[r] >= 0) {
            const float2* a = p.amp + (size_t)slot[r] * 6;
            vx += cmul_re(a[EX], pt0);
            vz += cmul_re(a[EZ], pt1);
            if (r < TY) vy += cmul_re(a[EY], pt0);
        }
        const bool z = G.zero(r);
        ex[r] = z ? 0.f : vx;
        ez[r] = z ? 0.f : vz;
        if (r < TY) ey[r] = z ? 0.f : vy;
    }
}

template <int TY, bool EDGE>
__device__ __forceinline__ void tile(const Problem& p, long long n, int par, int seg, int j0,
                                     int kb, int ke, int t) {
    const Geo<TY, EDGE> G(p, par, seg, j0);
    const int nz = p.nz, nx = p.nx, ny = p.ny;
    const int lane = threadIdx.x & 63;

    int slot[TY + 1];
#pragma unroll
    for (int r = 0; r <= TY; ++r) {
        slot[r] = -1;
        if (p.colmap && G.valid(r)) slot[r] = p.colmap[(size_t)G.jl[r + 1] * nx + G.xl];
    }

    // ---- prologue: E_new(kb) ------------------------------------------
    float hcx[TY], hcy[TY + 1], hcz[TY];      // H_old(k) kept for the H update
    float ecx[TY + 1], ecy[TY], ecz[TY + 1];  // E_new(k)
    {
        const int km = kb == 0 ? nz - 1 : kb - 1;
        float hx[TY + 2], hy[TY + 1], hz[TY + 2], hxm[TY], hym[TY + 1];
#pragma unroll
        for (int r = -1; r <= TY; ++r) {
            hx[r + 1] = G.ld(HX, kb, r);
            hz[r + 1] = G.ld(HZ, kb, r);
            if (r >= 0) {
                hy[r] = G.ld(HY, kb, r);
                hym[r] = G.ld(HY, km, r);
                ecx[r] = G.ld(EX, kb, r);
                ecz[r] = G.ld(EZ, kb, r);
            }
            if (r >= 0 && r < TY) {
                hxm[r] = G.ld(HX, km, r);
                ecy[r] = G.ld(EY, kb, r);
            }
        }
        e_plane<TY, EDGE>(G, n, kb, slot, hx, hy, hz, hxm, hym, ecx, ecy, ecz, true);
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            hcx[r] = hx[r + 1];
            hcy[r] = hy[r];
            hcz[r] = hz[r + 1];
        }
        hcy[TY] = hy[TY];
    }

    double en = 0.0;
    auto store_e = [&](int kk, const float (&ex)[TY + 1], const float (&ey)[TY],
                       const float (&ez)[TY + 1]) {
        if (!G.own_x) return;
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            if (!G.own_y(r)) continue;
            G.st(EX, kk, r, ex[r]);
            G.st(EY, kk, r, ey[r]);
            G.st(EZ, kk, r, ez[r]);
            if (p.epart) en += (double)ex[r] * ex[r] + (double)ey[r] * ey[r] + (double)ez[r] * ez[r];
            if (kk == p.plane) {
                const size_t pl = (size_t)G.jl[r + 1] * nx + G.xl, ps = (size_t)nx * ny;
                if (p.diag_mask & FDTD_DIAG_EX2) p.fl[pl] += (double)ex[r] * ex[r];
                if (p.diag_mask & FDTD_DIAG_EY2) p.fl[ps + pl] += (double)ey[r] * ey[r];
                if (p.diag_mask & FDTD_DIAG_EZ2) p.fl[2 * ps + pl] += (double)ez[r] * ez[r];
                if (p.rec) p.rec[(size_t)(n - p.rec_begin) * ps + pl] = ey[r];
            }
        }
    };
    store_e(kb, ecx, ecy, ecz);

    float hxb = 0.f, hxc = 0.f, hxk = 1.f;
    if (EDGE && G.xs >= 0) {
        hxb = cx_tab(p, T_HB)[G.xl];
        hxc = cx_tab(p, T_HC)[G.xl];
        hxk = cx_tab(p, T_HK)[G.xl];
    }
    const float2 th = p.colmap ? p.tH[n] : make_float2(0.f, 0.f);

    for (int k = kb; k < ke; ++k) {
        const int kn = k + 1 == nz ? 0 : k + 1;
        // ---- load H_old(k+1), E_old(k+1); form E_new(k+1) -------------
        float hx[TY + 2], hy[TY + 1], hz[TY + 2];
        float enx[TY + 1], eny[TY], enz[TY + 1];
#pragma unroll
        for (int r = -1; r <= TY; ++r) {
            hx[r + 1] = G.ld(HX, kn, r);
            hz[r + 1] = G.ld(HZ, kn, r);
            if (r >= 0) {
                hy[r] = G.ld(HY, kn, r);
                enx[r] = G.ld(EX, kn, r);
                enz[r] = G.ld(EZ, kn, r);
            }
            if (r >= 0 && r < TY) eny[r] = G.ld(EY, kn, r);
        }
        const bool own_next = k + 1 < ke;
        e_plane<TY, EDGE>(G, n, kn, slot, hx, hy, hz, hcx, hcy, enx, eny, enz, own_next);

        // ---- H_new(k) ---------------------------------------------------
        float2 qt0 = make_float2(0.f, 0.f), qt1 = qt0;
        if (p.colmap) {
            qt0 = cmul(p.zph[2 * k], th);
            qt1 = cmul(p.zph[2 * k + 1], th);
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const float ey_ip = __shfl_down(ecy[r], 1, 64);
            const float ez_ip = __shfl_down(ecz[r], 1, 64);
            float tyz = ecz[r + 1] - ecz[r];     // H_x: -(S_y Δ_y E_z
            const float dzey = eny[r] - ecy[r];  //        - S_z Δ_z E_y)
            const float dzex = enx[r] - ecx[r];  // H_y: -(S_z Δ_z E_x
            float txz = ez_ip - ecz[r];          //        - S_x Δ_x E_z)
            float txy = ey_ip - ecy[r];          // H_z: -(S_x Δ_x E_y
            float tyx = ecx[r + 1] - ecx[r];     //        - S_y Δ_y E_x)
            const bool own = G.own_x && G.own_y(r);
            if (EDGE) {
                if (G.xs >= 0) {
                    const size_t q = psix_at(p, k, G.jl[r + 1], G.xs);
                    float py = pptr(p, par, P_HYX)[q], pz = pptr(p, par, P_HZX)[q];
                    txz = cpml_term(txz, hxb, hxc, hxk, py, true);
                    txy = cpml_term(txy, hxb, hxc, hxk, pz, true);
                    if (own) {
                        pptr(p, par ^ 1, P_HYX)[q] = py;
                        pptr(p, par ^ 1, P_HZX)[q] = pz;
                    }
                }
                const int ys = G.ys[r + 1];
                if (ys >= 0) {
                    const int jr = G.jl[r + 1];
                    const float b = cy_tab(p, T_HB)[jr], c = cy_tab(p, T_HC)[jr];
                    const float kinv = cy_tab(p, T_HK)[jr];
                    const size_t q = psiy_at(p, k, ys, G.xl);
                    float px = pptr(p, par, P_HXY)[q], pz = pptr(p, par, P_HZY)[q];
                    tyz = cpml_term(tyz, b, c, kinv, px, true);
                    tyx = cpml_term(tyx, b, c, kinv, pz, true);
                    if (own) {
                        pptr(p, par ^ 1, P_HXY)[q] = px;
                        pptr(p, par ^ 1, P_HZY)[q] = pz;
                    }
                }
            }
            float vx = hcx[r] - (p.sy * tyz - p.sz * dzey);
            float vy = hcy[r] - (p.sz * dzex - p.sx * txz);
            float vz = hcz[r] - (p.sx * txy - p.sy * tyx);
            if (slot[r] >= 0) {
                const float2* a = p.amp + (size_t)slot[r] * 6;
                vx += cmul_re(a[HX], qt1);
                vy += cmul_re(a[HY], qt1);
                vz += cmul_re(a[HZ], qt0);
            }
            if (own) {
                G.st(HX, k, r, vx);
                G.st(HY, k, r, vy);
                G.st(HZ, k, r, vz);
                if (p.epart) en += (double)hcx[r] * vx + (double)hcy[r] * vy + (double)hcz[r] * vz;
            }
        }
        if (own_next) store_e(kn, enx, eny, enz);
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
    }
    if (p.epart) {
        en = wave_sum(en);
        if (lane == 0) p.epart[t] = en;
    }
}

// Tile decode and XCD-aware block remap shared by both launches.
struct TileIdx {
    int t, seg, sy, kb, ke;
};

__device__ __forceinline__ bool decode(int nsx, int nsy, int ncz, int cz, int nz,
                                       int nblocks_padded, TileIdx* ti) {
    // hardware block b runs on XCD b % 8; give each XCD a contiguous run
    const int b = blockIdx.x;
    const int lb = (b % 8) * (nblocks_padded / 8) + b / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = lb * WAVES_PER_BLOCK + wave;
    if (t >= nsx * nsy * ncz) return false;
    ti->t = t;
    ti->seg = t % nsx;
    ti->sy = (t / nsx) % nsy;
    const int czi = t / (nsx * nsy);
    ti->kb = czi * cz;
    ti->ke = min(ti->kb + cz, nz);
    return true;
}

// Interior tiles: every lane x in [max(npml,1), nx - npml), every row
// j0-1 .. j0+TY in [max(npml,1), ny - npml), no periodic wrap. They form the
// rectangle seg in [sx0, sx0+nsx), sy in [sy0, sy0+nsy) of the tile grid.
template <int TY>
__global__ void __launch_bounds__(64 * WAVES_PER_BLOCK)
fused_interior_kernel(Problem p, long long n, int par, int sx0, int sy0, int nsx, int nsy,
                      int ncz, int cz, int nblocks_padded, int nsx_all, int nsy_all) {
    TileIdx ti;
    if (!decode(nsx, nsy, ncz, cz, p.nz, nblocks_padded, &ti)) return;
    const int seg = sx0 + ti.seg, sy = sy0 + ti.sy;
    const int czi = ti.kb / cz;
    const int t = (czi * nsy_all + sy) * nsx_all + seg;   // global tile id (energy slot)
    tile<TY, false>(p, n, par, seg, sy * TY, ti.kb, ti.ke, t);
}

template <int TY>
__global__ void __launch_bounds__(64 * WAVES_PER_BLOCK)
fused_edge_kernel(Problem p, long long n, int par, int nsx, int nsy, int ncz, int cz,
                  int nblocks_padded, int sx0, int sx1, int sy0, int sy1) {
    TileIdx ti;
    if (!decode(nsx, nsy, ncz, cz, p.nz, nblocks_padded, &ti)) return;
    if (ti.seg >= sx0 && ti.seg < sx1 && ti.sy >= sy0 && ti.sy < sy1) return;   // interior
    tile<TY, true>(p, n, par, ti.seg, ti.sy * TY, ti.kb, ti.ke, ti.t);
}

int tiles(const Problem& p, int rows, int zchunk, int* nsx, int* nsy, int* ncz, int* cz) {
    *nsx = (p.nx + SEG - 1) / SEG;
    *nsy = (p.ny + rows - 1) / rows;
    *cz = zchunk > 0 ? zchunk : p.nz;
    *ncz = (p.nz + *cz - 1) / *cz;
    return *nsx * *nsy * *ncz;
}

}  // namespace

int fused_wave_count(const Problem& p, int rows, int zchunk) {
    int a, b, c, d;
    return tiles(p, rows, zchunk, &a, &b, &c, &d);
}

// Interior tile rectangle [sx0, sx1) × [sy0, sy1) (may be empty).
void interior_rect(const Problem& p, int rows, int nsx, int nsy, int* sx0, int* sx1, int* sy0,
                   int* sy1) {
    *sx0 = *sx1 = *sy0 = *sy1 = 0;
    if (p.periodic) return;
    const int m = p.npml > 0 ? p.npml : 1;
    // x: SEG*seg - 1 >= m and SEG*seg + 62 <= nx - npml - 1
    int a = (m + 1 + SEG - 1) / SEG;
    int b = (p.nx - p.npml - 1 - 62) >= 0 ? (p.nx - p.npml - 1 - 62) / SEG + 1 : 0;
    // y: rows*sy - 1 >= m and rows*sy + rows <= ny - npml - 1
    int c = (m + 1 + rows - 1) / rows;
    int d = (p.ny - p.npml - 1 - rows) >= 0 ? (p.ny - p.npml - 1 - rows) / rows + 1 : 0;
    b = min(b, nsx);
    d = min(d, nsy);
    if (a < b && c < d) {
        *sx0 = a; *sx1 = b; *sy0 = c; *sy1 = d;
    }
}

template <int TY>
hipError_t launch_rows(const Problem& p, long long n, int parity, int zchunk, hipStream_t s) {
    int nsx, nsy, ncz, cz;
    const int nt = tiles(p, TY, zchunk, &nsx, &nsy, &ncz, &cz);
    int sx0, sx1, sy0, sy1;
    interior_rect(p, TY, nsx, nsy, &sx0, &sx1, &sy0, &sy1);
    dim3 block(64 * WAVES_PER_BLOCK);
    const int ni = (sx1 - sx0) * (sy1 - sy0) * ncz;
    if (ni > 0) {
        const int nb = (ni + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        const int nbp = (nb + 7) / 8 * 8;
        hipLaunchKernelGGL(fused_interior_kernel<TY>, dim3(nbp), block, 0, s, p, n, parity, sx0,
                           sy0, sx1 - sx0, sy1 - sy0, ncz, cz, nbp, nsx, nsy);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ni < nt) {
        const int nb = (nt + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        const int nbp = (nb + 7) / 8 * 8;
        hipLaunchKernelGGL(fused_edge_kernel<TY>, dim3(nbp), block, 0, s, p, n, parity, nsx, nsy,
                           ncz, cz, nbp, sx0, sx1, sy0, sy1);
    }
    return hipGetLastError();
}

hipError_t launch_fused_step(const Problem& p, long long n, int parity, int rows, int zchunk,
                             hipStream_t s) {
    if (rows == 4) return launch_rows<4>(p, n, parity, zchunk, s);
    if (rows == 8) return launch_rows<8>(p, n, parity, zchunk, s);
    return hipErrorInvalidValue;
}

// Deterministic single-block sum of the per-wave energy partials.
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
