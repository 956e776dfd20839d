// Internal device-side layout of the gfx950 PIC library (not part of the ABI).
//
// Particles of one (box, species) live in SoA arrays binned by spatial tile.
// Two copies of the arrays alternate between steps: the push reads copy
// `cur` and writes every particle straight into the segment of its new tile in
// copy `cur ^ 1`, so the binning is refreshed every step at no extra traffic.
// Tile T owns the slots [seg_start[c][T], seg_start[c][T] + seg_cap[c][T]) of
// copy c and holds two ranges of particles there, all with their cell in T:
//   A = [0, na[c][T])                the tile's own particles that stayed,
//   B = [bs[c][T], bs[c][T] + nb[c][T])  particles that entered from elsewhere.
// The block that pushes tile T writes A from the front with an LDS counter and
// stages its leavers at the back of [0, n_src); at the end it hands them to
// the neighbouring tiles' B ranges, one global atomic per neighbour.  bs of the
// next step is the current particle count of the tile, set between steps.
// The last segment (index ntiles) is an overflow region (count nb[c][ntiles])
// for particles whose target range is full; it is swept by the slow path
// (fields read from HBM, current added with global atomics).  A counting-sort
// repack recomputes the segment layout from the actual counts.
//
// Stored particle state: cell packed as ix | iy << 11 | iz << 22, in-cell
// offset d in [0, 1) per axis, and u = gamma v / c.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

// Device pointers into the arena are global-memory pointers; saying so in the
// descriptor types lets the compiler emit global_* instead of flat_* memory
// instructions for every access through them.  The qualifier only exists in
// the device compilation of files with kernels; the host (and the host-only
// API file, which defines PIC_HOST_ONLY_TU) sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(PIC_HOST_ONLY_TU)
#define PIC_GLOBAL __attribute__((address_space(1)))
#else
#define PIC_GLOBAL
#endif

namespace pic {

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
constexpr int kOvfBlocks = 16;     // blocks per box sweeping the overflow region
constexpr int kBlock = 256;        // threads per block of the particle kernels
constexpr int kQBits = 31;         // fractional bits of the fixed-point current

__host__ __device__ inline int32_t pack_cell(int ix, int iy, int iz)
{
    return (int32_t)((uint32_t)ix | ((uint32_t)iy << 11) | ((uint32_t)iz << 22));
}
__host__ __device__ inline int cell_x(int32_t c) { return (int)((uint32_t)c & 2047u); }
__host__ __device__ inline int cell_y(int32_t c) { return (int)(((uint32_t)c >> 11) & 2047u); }
__host__ __device__ inline int cell_z(int32_t c) { return (int)((uint32_t)c >> 22); }

// A particle in a tile's ranges keeps its cell as a one-byte code local to
// the tile, x | y << tx | z << (tx + ty) (tile edges 2^tx, 2^ty, 2^tz, at most
// 256 cells; tiles start at multiples of their edges, so the code is the low
// bits of the cell's coordinates).  The overflow region, whose particles
// belong to any tile, and the leavers a push stages for the hand-over keep the
// packed cell.
template <typename R>
struct PBuf {                      // one copy of the particle arrays
    PIC_GLOBAL uint8_t *lc;        // tile-local cell code (tile ranges); nullptr in the stage
    PIC_GLOBAL int32_t *cell;      // packed cell (overflow region, staged leavers, stage)
    PIC_GLOBAL R *d[3];
    PIC_GLOBAL R *u[3];
    PIC_GLOBAL int32_t *id;        // nullptr without PIC_TRACK_IDS
};

template <typename R>
struct SpeciesDev {
    PBuf<R> buf[2];
    PBuf<R> stage;                 // freshly loaded / set particles, unbinned
    PIC_GLOBAL int32_t *seg_start[2];   // ntiles + 1 per copy (last: overflow region)
    PIC_GLOBAL int32_t *seg_cap[2];     // ntiles + 1 per copy
    PIC_GLOBAL int32_t *na[2];          // ntiles + 1 per copy: A-range count
    PIC_GLOBAL int32_t *nb[2];          // ntiles + 1 per copy: B-range count (overflow count last)
    PIC_GLOBAL int32_t *bs[2];          // ntiles + 1 per copy: B-range start
    PIC_GLOBAL int32_t *tcount;         // ntiles + 1, repack scratch
    int32_t slots;                 // length of each array
    int32_t ovf_cap;               // slots reserved for the overflow region
};

// J type: int64 fixed point (2^-31 cell volumes) for FP32, double for FP64.
template <typename R> struct JType;
template <> struct JType<float> { using T = long long; };
template <> struct JType<double> { using T = double; };

template <typename R>
struct BoxDev {
    int32_t n[3];
    int32_t tshift[3];             // log2 of the tile edge per axis
    int32_t ntile[3];
    int32_t ntiles;
    int64_t nc;
    PIC_GLOBAL R *e;               // 3 * nc, e^t
    PIC_GLOBAL R *b;               // 3 * nc, b^{t-dt/2}
    PIC_GLOBAL R *bn;              // 3 * nc, the other b buffer: the push writes b^{t+dt/2} there
    PIC_GLOBAL typename JType<R>::T *J;   // 3 * nc, current of the step in flight
    PIC_GLOBAL double *rho;        // nc, diagnostic charge density
    PIC_GLOBAL double *acc;        // diagnostic accumulators (kAccLen doubles)
    PIC_GLOBAL int64_t *hist;      // n_species * hist_bins
    double alpha0;                 // 2 / (n_x^2 rho0)
    int32_t wall;                  // axis with conducting walls, -1: periodic
    int32_t faraday4;              // fourth-order curl of e in Faraday's law
    SpeciesDev<R> sp[kMaxSpecies];
};

// per-launch constants of the particle kernels
template <typename R>
struct StepConst {
    R dt;
    int32_t nsp;
    R kq[kMaxSpecies];             // (q/e)(m_e/m)
    R qs[kMaxSpecies];             // sgn(q)
    R mass[kMaxSpecies];           // m/m_e
    PIC_GLOBAL uint32_t *flags;    // device error flag word
    int32_t cur;                   // copy read this step
    int32_t hist_bins;
    double hist_lo, hist_hi;
    int32_t filter;                // smooth the current (and the Gauss charge)
};

// diagnostic accumulator layout per box
constexpr int kAccField = 0;       // [0..2] sum e^2/2, [3..5] sum (b^t)^2/2, [6] gauss max, [7] gauss sum sq
constexpr int kAccSp = 8;          // then per species 6: K, P[3], count, sum(gamma-1)
constexpr int kAccLen = kAccSp + 6 * kMaxSpecies;

// work item of the particle kernels: box, and tile (>= 0) or -1-k for overflow
// block k; box -1 is an idle item (padding of the push order)
struct Item {
    int32_t box;
    int32_t tile;
};

__device__ inline int wrap_idx(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <typename R>
__device__ inline int tile_of(const BoxDev<R> &B, int32_t c)
{
    // tile counts are below 2^11, so 24-bit multiplies are exact
    const unsigned ty = (unsigned)(cell_y(c) >> B.tshift[1]), tz = (unsigned)(cell_z(c) >> B.tshift[2]);
    return (cell_x(c) >> B.tshift[0]) +
           (int)__umul24((unsigned)B.ntile[0], ty + __umul24((unsigned)B.ntile[1], tz));
}

// Tile-local code of a cell (the low bits of its coordinates) and its inverse
// for a tile with origin o.
template <typename R>
__device__ inline int local_code(const BoxDev<R> &B, int32_t c)
{
    const int sx = B.tshift[0], sy = B.tshift[1];
    return (cell_x(c) & ((1 << sx) - 1)) | ((cell_y(c) & ((1 << sy) - 1)) << sx) |
           ((cell_z(c) & ((1 << B.tshift[2]) - 1)) << (sx + sy));
}

template <typename R>
__host__ __device__ inline int32_t local_cell(const BoxDev<R> &B, const int o[3], int code)
{
    const int sx = B.tshift[0], sy = B.tshift[1];
    return pack_cell(o[0] + (code & ((1 << sx) - 1)), o[1] + ((code >> sx) & ((1 << sy) - 1)), o[2] + (code >> (sx + sy)));
}

// Origin cell of tile T.
template <typename R>
__host__ __device__ inline void tile_origin(const BoxDev<R> &B, int T, int o[3])
{
    const int r = T / B.ntile[0];
    o[0] = (T - r * B.ntile[0]) << B.tshift[0];
    o[1] = (r % B.ntile[1]) << B.tshift[1];
    o[2] = (r / B.ntile[1]) << B.tshift[2];
}

// cell blocks of the field kernels: (box, first cell) of kBlock cells
struct CellBlock {
    int32_t box;
    int32_t first;
};

// stage item: particles [first, last) of the stage of (box, species); half:
// integrate their momenta back by dt/2 when they are binned
struct StageItem {
    int32_t box, species, first, last, half;
};

// one drifting Maxwell-Juttner population of a load
struct MJPop {
    double mu, G, beta0;
    int axis;
    const PIC_GLOBAL double *tab;
};

struct LoadArgs {
    int32_t box, sa, sb;
    int64_t npairs;
    int32_t offa, offb;        // first stage slot of each species
    int32_t ida, idb;          // first particle id of each species
    int32_t profile, paxis;
    double centre, thick, halfw;
    uint64_t seed, stream;
    int N;                     // table intervals
    MJPop A, B;
};

// Where the diagnostics sum: kAccLen accumulators, the charge density (one
// value per cell) and the gamma-1 histogram (n_species x bins).  pic_diag
// points it into the arena, pic_diag_noalloc into the library's static
// scratch.
struct DiagBuf {
    PIC_GLOBAL double *acc;
    PIC_GLOBAL double *rho;
    PIC_GLOBAL int64_t *hist;
};

// size of the static scratch of pic_diag_noalloc (per GPU)
constexpr size_t kDiagScratchBytes = size_t(32) << 20;

// launchers (pic_kernels.hip, pic_loader.hip)
template <typename R> size_t push_lds_bytes(int t0, int t1, int t2);
template <typename R>
hipError_t launch_push(const BoxDev<R> *boxes, const Item *items, int nitems, size_t lds, const StepConst<R> &C,
                       int fixed444, int walls, int faraday4, hipStream_t st);
template <typename R>
hipError_t launch_fields(const BoxDev<R> *boxes, const CellBlock *blocks, int nblocks, R dt, int nsp, int filter,
                         int clear_copy, int nboxes, uint32_t *watch, hipStream_t st);
template <typename R>
hipError_t launch_advance_b(const BoxDev<R> *boxes, const CellBlock *blocks, int nblocks, R h, hipStream_t st);
template <typename R>
hipError_t launch_repack(const BoxDev<R> *boxes, int nboxes, const Item *items, int nitems,
                         const StageItem *sitems, int nsitems, const StepConst<R> &C, hipStream_t st);
template <typename R>
hipError_t launch_diag(const BoxDev<R> *boxes, int box, int64_t nc, const Item *items, int nitems,
                       const StepConst<R> &C, const DiagBuf &out, int hist_len, hipStream_t st);
// device address of the static diagnostics scratch of the current device:
// set up once per device (pic_init), then read
hipError_t diag_scratch_setup();
void *diag_scratch();
hipError_t launch_mj_table(double theta, double gamma_beta, double *cum, int M, int N, double *tab,
                           hipStream_t st);
template <typename R> hipError_t launch_load_pairs(const BoxDev<R> *boxes, const LoadArgs &L, hipStream_t st);
template <typename R>
hipError_t launch_harris_field(const BoxDev<R> *boxes, int64_t nc, const pic_harris_field &H, hipStream_t st);
template <typename R>
hipError_t launch_spectrum(const BoxDev<R> *boxes, int box, const int n[3], int f, int c, int an, R hdt,
                           double *scratch, double *ps, hipStream_t st);

} // namespace pic
