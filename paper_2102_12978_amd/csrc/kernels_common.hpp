// Device helpers shared by the Yee kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "fdtd_internal.hpp"

// Automatic contraction off for every file that includes this header (the
// kernels): fused multiply-adds only where the helpers below ask for them.
#pragma clang fp contract(off)

namespace bfdtd {

// Every pointer in a Problem addresses device global memory. A Problem read
// from memory (the batched kernels) holds them as generic pointers, which the
// compiler would access with flat instructions; the accessors below return
// them cast to the global address space, so every kernel emits global loads
// and stores whichever way its Problem arrived.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> G(T* q) {
    return (gptr<T>)q;
}

// float2 element i of a global array (HIP's float2 class cannot be copied
// out of the global address space directly; one 8-byte load).
__device__ __forceinline__ float2 ld2(gptr<const float2> q, size_t i) {
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = ((gptr<const v2f>)q)[i];
    return make_float2(v.x, v.y);
}

// float2 element i of a table no kernel writes (the z phases e^{iβz}, the
// time factors), read through the constant address space: with a
// wavefront-uniform index that is a scalar load, whose wait leaves the
// vector-memory counter, and so the wavefront's field loads and stores in
// flight, alone. A lane-varying index still gives a vector load.
template <typename T>
using cptr = __attribute__((address_space(4))) const T*;

__device__ __forceinline__ float2 ldc2(const float2* q, size_t i) {
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = ((cptr<v2f>)q)[i];
    return make_float2(v.x, v.y);
}

// CPML slab index of an x position (-1 outside the slabs).
__device__ __forceinline__ int slab_index(int i, int n, int npml) {
    if (npml <= 0) return -1;
    if (i < npml) return i;
    if (i >= n - npml) return i - n + 2 * npml;
    return -1;
}

__device__ __forceinline__ size_t psix_at(const Problem& p, int k, int j, int xs) {
    return ((size_t)k * p.ny + j) * (2 * p.npml) + xs;
}

__device__ __forceinline__ size_t psiy_at(const Problem& p, int k, int ys, int i) {
    return ((size_t)k * (2 * p.npml) + ys) * p.pitch + i;
}

__device__ __forceinline__ gptr<float> fptr(const Problem& p, int par, int c) {
    return G(p.fbase[par]) + c * p.fstride;
}

__device__ __forceinline__ gptr<float> pptr(const Problem& p, int par, int q) {
    return G(p.pbase[par]) + psi_offset(p, q);
}

__device__ __forceinline__ gptr<const float> cx_tab(const Problem& p, int t) {
    return G(p.ctab) + (size_t)t * p.nx;
}

__device__ __forceinline__ gptr<const float> cy_tab(const Problem& p, int t) {
    return G(p.ctab) + (size_t)6 * p.nx + (size_t)t * p.ny;
}

// The terms of the cell updates, each with its roundings fixed by an explicit
// fused multiply-add. Every Yee kernel (one-step, two-step, frame, batch)
// forms a cell from these, in files compiled with automatic contraction
// off, so that all of them round a cell alike and their states agree bit
// for bit whatever the compiler would otherwise fuse.
//   a·x − b·y      (a curl pair: S_d Δ_d u − S_e Δ_e v)
__device__ __forceinline__ float curl_pair(float a, float x, float b, float y) {
    return __builtin_fmaf(a, x, -(b * y));
}
//   b·ψ + c·Δ      (CPML memory update)
__device__ __forceinline__ float cpml_mem(float b, float psi, float c, float d) {
    return __builtin_fmaf(b, psi, c * d);
}
//   k·Δ + ψ        (stretched difference: Δ/κ + ψ)
__device__ __forceinline__ float stretched(float kinv, float d, float psi) {
    return __builtin_fmaf(kinv, d, psi);
}
//   acc + v²       (plane and energy sums, FP64)
__device__ __forceinline__ double sq_acc(double acc, float v) {
    return __builtin_fma((double)v, (double)v, acc);
}

// Re{a · b}
__device__ __forceinline__ float cmul_re(float2 a, float2 b) {
    return __builtin_fmaf(a.x, b.x, -(a.y * b.y));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// Column c of the frame -> (x, y). A plane holds fewer than 2^31 cells (the
// context checks it), so the index math is 32-bit: unsigned divisions are a
// fraction of the cost of 64-bit ones.
__device__ __forceinline__ bool frame_column(const Frame& fr, int nx, int ny, unsigned c, int* x,
                                             int* y) {
    const unsigned unx = (unsigned)nx;
    const unsigned nb = (unsigned)fr.y0 * unx;
    const unsigned nt = (unsigned)(ny - fr.y1) * unx;
    const unsigned nl = (unsigned)(fr.y1 - fr.y0) * (unsigned)fr.x0;
    const unsigned nr = (unsigned)(fr.y1 - fr.y0) * (unsigned)(nx - fr.x1);
    if (c < nb) {
        *y = (int)(c / unx);
        *x = (int)(c % unx);
    } else if ((c -= nb) < nt) {
        *y = fr.y1 + (int)(c / unx);
        *x = (int)(c % unx);
    } else if ((c -= nt) < nl) {
        *y = fr.y0 + (int)(c / (unsigned)fr.x0);
        *x = (int)(c % (unsigned)fr.x0);
    } else if ((c -= nl) < nr) {
        const unsigned wdt = (unsigned)(nx - fr.x1);
        *y = fr.y0 + (int)(c / wdt);
        *x = fr.x1 + (int)(c % wdt);
    } else {
        return false;
    }
    return true;
}

// Sum over a wave64 (deterministic butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace bfdtd
