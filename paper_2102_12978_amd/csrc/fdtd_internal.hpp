// Internal types shared by the host set-up, the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fdtd.h"

namespace bfdtd {

enum { EX = 0, EY, EZ, HX, HY, HZ };
// CPML memories: ψ of (component, derivative axis)
enum { P_EXY = 0, P_EYX, P_EZX, P_EZY, P_HXY, P_HYX, P_HZX, P_HZY };
// 1-D CPML tables: b, c, 1/κ at integer (E) and half-integer (H) positions
enum { T_EB = 0, T_EC, T_EK, T_HB, T_HC, T_HK };

// Everything a kernel needs to advance one problem instance. Plain data,
// passed by value to single-domain launches and read from device memory by
// the batched persistent kernel. Few pointers on purpose: every field of one
// parity lives in one allocation (component c at fbase[par] + c*fstride), the
// eight CPML memories of one parity in another (x-slab arrays first), and
// the twelve CPML coefficient rows in a third.
struct Problem {
    int nx, ny, nz, pitch;          // pitch: floats per x row
    int npml;                       // CPML cells (0: none)
    int periodic;                   // x/y periodic test mode
    int plane;                      // diagnostic plane, -1: none
    int diag_mask;                  // FDTD_DIAG_* bits accumulated this step
    float sx, sy, sz;               // S Δx/Δ_d
    int n_slots;
    float* fbase[2];                // ping-pong fields [parity]
    long long fstride;              // floats per component (nz*ny*pitch)
    float* pbase[2];                // ping-pong CPML memories [parity]
    long long psx;                  // floats per x-slab array (nz*ny*2*npml)
    long long psy;                  // floats per y-slab array (nz*2*npml*pitch)
    const float* ctab;              // [6][nx] x tables then [6][ny] y tables
    const int* colmap;              // [ny][nx] antenna slot or -1
    const float2* amp;              // [slot][6] w·Ã (FP32 from FP64)
    const float2* zph;              // [nz][2] e^{iβ z} at integer / half planes
    const float2* tE;               // [step] f(t_{n+1}) e^{-iω(t_{n+1}-T0)}
    const float2* tH;               // [step] f(t_{n+3/2}) e^{-iω(t_{n+3/2}-T0)}
    double* fl;                     // [3][ny][nx] plane sums (E_x², E_y², E_z²)
    float* rec;                     // E_y plane record (adjoint), or null
    long long rec_begin;            // first recorded step
    long long win_begin;            // batched kernels: first step whose plane is accumulated
};

// Position of CPML memory q (P_* order) inside one parity's allocation.
__host__ __device__ inline long long psi_offset(const Problem& p, int q) {
    switch (q) {
        case P_EYX: return 0;
        case P_EZX: return p.psx;
        case P_HYX: return 2 * p.psx;
        case P_HZX: return 3 * p.psx;
        case P_EXY: return 4 * p.psx;
        case P_EZY: return 4 * p.psx + p.psy;
        case P_HXY: return 4 * p.psx + 2 * p.psy;
        default:    return 4 * p.psx + 3 * p.psy;   // P_HZY
    }
}

inline size_t field_elems(const Problem& p) { return (size_t)p.nz * p.ny * p.pitch; }
inline size_t psix_elems(const Problem& p) { return (size_t)p.nz * p.ny * 2 * p.npml; }
inline size_t psiy_elems(const Problem& p) { return (size_t)p.nz * 2 * p.npml * p.pitch; }
inline size_t psi_total(const Problem& p) { return 4 * psix_elems(p) + 4 * psiy_elems(p); }

// Host-side antenna description (double precision).
struct Antenna {
    double k = 0, beta = 0, kr = 0, omega = 0, t0 = 0;
    int ramp_kind = FDTD_RAMP_SIN2;
    double ramp_a = 0, ramp_b = 0;       // normalised time units
    double e0 = 1;
    int order = 0;
    int polarization = FDTD_POL_X_TE;
    double theta = 0;
    double ax = 0, ay = 0, r_in = 0, r_out = 0;
    int n_sectors = 0;
    std::vector<double> sec_amp, sec_phase;
    // per slot: column and, per component, base amplitude and sector
    std::vector<int> slot_i, slot_j;
    std::vector<double> base_re, base_im;   // [slot*6 + c]
    std::vector<int> member;                // [slot*6 + c] 1 if a source point
    std::vector<int> sector;                // [slot*6 + c]
    int n_source[6] = {0, 0, 0, 0, 0, 0};
};

// Time factor f(t) e^{-iω(t - T0)} in double precision.
void time_factor(const Antenna& a, double t, double* re, double* im);

// Build the antenna (membership, amplitudes) for a grid. Returns an error
// message or empty on success.
std::string build_antenna(const fdtd_grid& g, int pitch, double ry, double rz,
                          const fdtd_injector& inj, Antenna* out);

// Weighted FP32 amplitudes [slot][6] as interleaved (re, im).
void weighted_amplitudes(const Antenna& a, std::vector<float>* out);

// CPML 1-D tables (b, c, 1/κ) at E and H positions along one axis.
void cpml_axis_tables(int n, int npml, double delta_ratio, const fdtd_grid& g, double dt,
                      std::vector<float>* tabs /* 6 vectors of n */);

std::string validate_grid(const fdtd_grid& g);

// Optional per-launch timing: launchers call mark(name) before each kernel
// and mark(nullptr) after the last one, on the timer's own stream; a
// launcher that spreads kernels over several streams brackets each one with
// mark_on(name, s) and mark_on(nullptr, s) on that kernel's stream.
struct LaunchTimer {
    virtual void mark(const char* name) = 0;
    virtual void mark_on(const char* name, hipStream_t s) = 0;
    virtual ~LaunchTimer() {}
};

// Rectangle of cells [x0, x1) × [y0, y1) that the split kernels leave out
// (all zero: the split kernels cover the whole grid).
struct Frame {
    int x0, x1, y0, y1;
};

// Fused interior kernel (kernels_fused.hip); rows per wavefront: 4 or 8;
// xalign: the interior starts on a multiple of 32 or 64 cells in x.
Frame fused_interior_rect(const Problem& p, int rows, int xalign);
int fused_interior_tiles(const Problem& p, int rows, int zchunk, int xalign);
// z chunk giving the interior kernel about 32 workgroups per CU (at least 4
// planes per chunk; 0: the whole z already gives that many)
int fused_default_zchunk(const Problem& p, int rows, int xalign, int cus);
hipError_t launch_fused_interior(const Problem& p, long long n, int parity, int rows, int zchunk,
                                 int xalign, double* epart, hipStream_t s, LaunchTimer* timer);

// Split kernels over the frame around a rectangle (kernels_split.hip)
long long frame_columns(const Problem& p, const Frame& fr);
int split_partial_count(const Problem& p, const Frame& fr);
hipError_t launch_split_frame(const Problem& p, long long n, int parity, const Frame& fr,
                              double* epart, hipStream_t s, LaunchTimer* timer);

// Two-step kernel over the whole grid (kernels_step2.hip); rows per
// wavefront 2 or 4; zchunk 0: the whole z. One call advances fields and CPML
// memories from parity `parity` at step n to parity ^ 1 at step n + 2
// (mask0 / mask1: plane accumulation of steps n and n + 1) in four launches
// (interior, x boundary, y boundary and corner tiles), the boundary ones on
// the side streams when given (and no timer is attached). Not for the
// periodic test mode.
struct SideStreams {
    hipStream_t s[3];               // default-priority streams beside the caller's
    hipEvent_t fork, join[3];       // timing-disabled events
};
hipError_t launch_step2(const Problem& p, long long n, int parity, int rows, int zchunk,
                        int mask0, int mask1, hipStream_t s, LaunchTimer* timer,
                        const SideStreams* side);
// Cells (times nz) of the interior-class launch: tiles with no wall or CPML
long long step2_interior_cells(const Problem& p, int rows);
// The three-step kernel (kernels_step3.hip): as launch_step2 with a third
// step, from parity `parity` at step n to parity ^ 1 at step n + 3 (mask0..2:
// plane accumulation of steps n .. n + 2), in the same four tile classes
// (58-cell x segments). Not for the periodic test mode.
hipError_t launch_step3(const Problem& p, long long n, int parity, int rows, int zchunk,
                        int mask0, int mask1, int mask2, hipStream_t s, LaunchTimer* timer,
                        const SideStreams* side);
long long step3_interior_cells(const Problem& p, int rows);
// The two-step kernel over many instances: work items (instance, segment,
// row group, kb | ke << 16) per tile class (0 interior, 1 x boundary, 2 y
// boundary, 3 corner; nz < 65536), and one pair of steps of every instance
// (four launches, step index *nctr + off, parity par; diag: plane
// accumulation as each Problem selects from its window on). With side
// streams the boundary classes run beside the interior one, forked from and
// joined back into s (also under stream capture); without, all on s.
void step2_batch_items(const std::vector<Problem>& probs, int rows, int zchunk,
                       std::vector<int4> items[4]);
hipError_t launch_step2_batch(const Problem* probs, const int4* const items[4],
                              const int nitems[4], int rows, const long long* nctr, int off,
                              int par, int diag, hipStream_t s, const SideStreams* side);

hipError_t launch_energy_reduce(const double* part, int n, double* out, hipStream_t s);

// Batched kernels over many instances (kernels_batch.hip). A work item is
// (instance, first flattened column, k begin, k end); with planes == 0 the E
// and H kernels loop over the items with a persistent grid of `blocks`
// workgroups of `cols` threads; with planes > 0 they launch one workgroup per
// (item, plane < planes) and ignore the items' k range. The step index is
// *nctr + off (a device counter so that a captured graph can be replayed);
// par is the parity read.
hipError_t launch_batch_e(const Problem* probs, const int4* work, int nwork, int cols, int blocks,
                          int planes, const long long* nctr, int off, int par, int diag,
                          hipStream_t s);
hipError_t launch_batch_h(const Problem* probs, const int4* work, int nwork, int cols, int blocks,
                          int planes, const long long* nctr, int off, int par, hipStream_t s);
hipError_t launch_batch_advance(long long* nctr, int by, hipStream_t s);
int batch_blocks_per_cu(int cols);   // resident workgroups per CU of both batch kernels

// Fused step over boundary tiles (kernels_fused_bnd.hip): tiles (instance,
// x0, y0, z chunk of cz planes) of 64 x cells by rows (2 or 4) rows, of
// probs[instance], or of `single` when probs is null; cells inside excl are
// not stored. Step index *nctr + n_off (nctr may be null). epart: one
// partial per tile, or null.
hipError_t launch_fused_bnd(const Problem& single, const Problem* probs, const int4* tiles,
                            int ntiles, int rows, int cz, int blocks, const long long* nctr,
                            long long n_off, int par, int diag, const Frame& excl, double* epart,
                            hipStream_t s);
int fused_bnd_blocks_per_cu(int rows, bool multi);

}  // namespace bfdtd
