// Device-side layout of one simulation and the helpers shared by the kernels.
//
// Grid: nx x ny cells.  Storage is row-major with x fastest; with the moving
// window the x axis is a ring of nxs >= nx + TX + 2 columns in which window
// column w lives at storage column (origin + w) mod nxs and the other
// nxs - nx columns (the "gap") are held at zero.  The gap is wider than a tile
// plus its guard cells, so no tile's halo ever sees both window edges.
//
// Tiles: TX x TY cells (the paper's regions with ghost cells, Sec. 3.2).  A
// tile owns a segment of particle slots per species and buffer (see SpDev),
// of which the first count[t] are live.  Fields and current are staged per tile in LDS on
// local cells [-1, TX+2) x [-1, TY+2): one guard cell below and two above,
// which is the reach of bilinear interpolation of the staggered components
// (one cell each way) and of the charge-conserving deposit of a particle that
// moves at most one cell per step (two cells up).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int TX = 16;
constexpr int TY = 16;
constexpr int PX = TX + 3;          // LDS row pitch of a tile block
constexpr int PY = TY + 3;
constexpr int BP = PX * PY;         // cells of a tile block
constexpr int NT = 256;             // threads per block (4 wavefronts)
constexpr int NTP = 512;            // threads per push block (8 wavefronts)
constexpr int NTP_BIG = 1024;       // ... for tiles loaded with >= BIG_TILE particles
constexpr int BIG_TILE = 65536;
constexpr int NTB = 512;            // threads per batched push block
constexpr int MAX_SP = 4;
constexpr int MAX_FR = 4;
// Streaming field kernels: the fold takes half a tile row (FH rows) of four
// tiles per wavefront, the filter + Yee a strip of YS_S rows and
// yee_strip_w(rf) columns (rf = filter passes + compensator).
constexpr int FH = 8;
constexpr int YS_S = 6;
__host__ __device__ constexpr int yee_strip_w(int rf) { return 63 - 2 * (rf > 1 ? rf : 1); }
__host__ __device__ constexpr int fold_units(int ntx, int nty) { return ((ntx + 3) / 4) * nty * 2; }
__host__ __device__ constexpr int yee_units(int nxs, int ny, int rf)
{
    return ((nxs + yee_strip_w(rf) - 1) / yee_strip_w(rf)) * ((ny + YS_S - 1) / YS_S);
}           // largest filter halo (passes + compensator)
constexpr int QX = TX + 2 * MAX_FR; // LDS pitch of the filter block
constexpr int QY = TY + 2 * MAX_FR;
// Device error bits (DevState::err): which store ran out of slots.
constexpr int ERR_SEG = 1;         // a tile's segment (push output)
constexpr int ERR_OUTBOX = 2;      // a tile's outbox
constexpr int ERR_ARRIVALS = 4;    // a push block's arrival list
constexpr int ERR_SETTLE = 8;      // a segment while appending pending leavers
constexpr int ERR_POOL = 16;       // the pool, for a relayout's needs
constexpr int ERR_INJECT = 32;     // a segment while loading the window's new column
constexpr int ERR_LOAD = 64;       // a segment during the initial load
constexpr int ERR_CAPACITY = 127;  // any of them
constexpr int N_RED = 16;           // result slots of the diagnostic reduction
constexpr int NB_DIAG = 512;        // blocks of the grid-stride diagnostic kernels

// Mutable per-simulation state read by every kernel of a step, so that one
// captured step graph can be replayed.
struct DevState {
    long long iter;   // completed steps
    int parity;       // field buffer holding E^n, B^n
    int origin;       // storage column of window column 0
    int nshift;       // window shifts done
    int shift;        // 1 if the last step shifted the window
    int err;          // ERR_* bits
    int ppar;         // particle buffer holding the tiles' particles
    int opar;         // outbox written by the last push
    int pend;         // 1: that outbox holds leavers not yet in any tile
    int blocks_done;  // blocks of the running push launch that finished
    int relay;        // 1: a push left some tile's segment short (relayout at the step end)
};

// Particle hand-off between tiles.  A push reads its tile from particle
// buffer ppar, together with the leavers its 8 neighbours sent it in outbox
// opar (if pending), and writes the particles that stay, compacted, to buffer
// ppar ^ 1 and the ones that leave to outbox opar ^ 1, each tagged with the
// direction (dx, dy) of its tile step; the neighbour in that direction picks
// it up.  The launch's last block to finish then flips both parities and
// marks the new outbox pending; k_settle appends pending leavers to their tiles when the particle
// set must be complete (host reads, diagnostics, window shifts).
constexpr int N_DIR = 8;
__device__ __forceinline__ int dir_index(int dtx, int dty)
{
    const int k = (dtx + 1) + 3 * (dty + 1);  // 0..8 without the centre 4
    return k < 4 ? k : k - 1;
}

template <typename R>
struct PartBuf {
    int *cell;        // packed storage cell: ix | iy << 16 (16 bits each, unsigned)
    R *x, *y, *ux, *uy, *uz;
    int *count;       // particles per tile
};

// Particle storage of a species: two ping-pong buffers of `pool` slots in
// which tile t owns the segment [start[b][t], start[b][t] + seg[b][t]) of
// buffer b, its particles in the first count[t] slots.  Segments are sized
// per tile from the particle counts (a relayout every few steps gives each
// tile room for its count plus twice its growth since the last check, and
// shares the rest of the pool in proportion to count + average), so a tile
// holding several times the average load needs no uniform over-sizing.
// The push reads its tile from buffer b and writes it to buffer b ^ 1 at the
// latter's layout, so a new layout costs nothing beyond that push.
template <typename R>
struct SpDev {
    PartBuf<R> pb[2];                 // ping-pong particle buffers of `pool` slots
    long long *start[2];              // per buffer: first slot of each tile's segment
    int *seg[2];                      // per buffer: slots of each tile's segment
    int *snap;                        // each tile's count at the last layout check
    int *need;                        // each tile's need at the check (scratch)
    int *inflow;                      // particles that entered each tile in its
                                      // last step with a hand-off
    int *ob_cell[2];                  // outboxes: ntiles x cap_out
    R *ob_x[2], *ob_y[2], *ob_ux[2], *ob_uy[2], *ob_uz[2];
    unsigned char *ob_dir[2];         // dir_index of each leaver's tile step
    int *ob_count[2];                 // leavers per tile
    R qm, qp, tau;    // q/m, charge per particle, (dt/2)(q/m)
    long long pool;   // slots per buffer
    int maxseg;       // most slots one tile's segment may have
    int ppc_x, ppc_y;
    double density, x_lo, x_hi;
    double uth[3], ufl[3];
};

template <typename R>
struct SimDev {
    int nx, ny, nxs;
    int ntx, nty, ntiles;
    int rx, ry;       // tiles the fold searches on each side along x, y: 1, or 2
                      // where the last tile is one cell wide (see fold_reach)
    int window, nsp, cap_out;
    int push_bt;      // threads per single-simulation push block: NTP or NTP_BIG
    int nsb;          // push blocks per tile: 1, or one per species (blk then holds
                      // nsb slices of 64-bit sums per tile)
    int *order;       // work items of the single-simulation push (ntiles * nsb):
                      // block b takes order[b]; heaviest first
    int npass, compensate;
    int direct;       // 1: colour-phased deposit straight into J (no fold)
    R dx, dy, dt;
    R idx, idy;       // 1/dx, 1/dy
    R dt_dx, dt_dy;   // dt/dx, dt/dy
    R jxs, jys;       // dx/dt, dy/dt
    double dx_d, dy_d, dt_d;
    R jq;             // fixed-point scale: 2^(e-32) in FP32, 2^e in FP64
    double jq_inv;    // 2^-e, value of one unit of an LDS sum
    unsigned key0, key1;
    R *F[2][6];       // ping-pong Ex Ey Ez Bx By Bz
    R *J[3];          // folded current of the last step
    R *Jf[3];         // filtered current (aliases J without a filter)
    R *blk;           // per-tile current blocks: ntiles x 3 x BP
    R *rho, *rho_f, *rho_prev;
    double *g0;       // div E^0 - F rho^0
    double *red;      // reduction partials
    double *res;      // N_RED reduced results
    DevState *st;
    SpDev<R> sp[MAX_SP];
};

__device__ __forceinline__ int wrapi(int a, int n)
{
    a += (a < 0) ? n : 0;
    a -= (a >= n) ? n : 0;
    return a;
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run
// of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Current and charge are summed in LDS as 64-bit fixed point: integer LDS
// atomics run at the rate of plain LDS traffic on CDNA, floating-point ones
// do not, and integer sums do not depend on the order of the additions, so
// the result is bitwise reproducible.  A term v enters as v * 2^e made an
// integer (FP32: floor; FP64: nearest).
// Callers pass y = v * jq with the power-of-two scale jq folded into their
// per-species prefactors, so y rounds exactly as v would.  FP32 (jq =
// 2^(e-32)): the high word is floor(y) and the low word fract(y) * 2^32, both
// exact; the hardware fract is clamped below 1, which moves a negative term
// smaller than 2^-25 in y by less than 2^-24 in y.  FP64 (jq = 2^e): y rounded
// to the nearest integer.
__device__ __forceinline__ void lds_acc(unsigned long long *p, float y)
{
    int hi;  // floor(y) converted in one instruction
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(hi) : "v"(y));
    const unsigned lo = (unsigned)(__builtin_amdgcn_fractf(y) * 4294967296.0f);
    const unsigned long long q = ((unsigned long long)(unsigned)hi << 32) | lo;
    __hip_atomic_fetch_add(p, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_acc(unsigned long long *p, double y)
{
    // nearest integer: a floor would lower every term by half a unit on
    // average, and an entry that sums thousands of terms would drift by as
    // many half-units
    const long long q = (long long)rint(y);
    __hip_atomic_fetch_add(p, (unsigned long long)q, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Pointers in the descriptors are generic; every array they reach is in
// device memory.  Pointers loaded from a descriptor table in memory (the
// batched kernels) cannot be proven global by the compiler, which then emits
// flat accesses with 64-bit vector addresses; glob() states the address space.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> glob(T *p)
{
    return (gptr<T>)p;
}

// Tile t's segment of buffer b: first slot and slots.
template <typename R>
__device__ __forceinline__ size_t seg_start(const SpDev<R> &P, int b, int t)
{
    return (size_t)glob(P.start[b])[t];
}
template <typename R>
__device__ __forceinline__ int seg_slots(const SpDev<R> &P, int b, int t)
{
    return glob(P.seg[b])[t];
}

// element at a 32-bit byte offset from a wave-uniform base pointer (keeps the
// address computation in 32 bits: base in SGPRs, offset in one VGPR)
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T &at(T *base, unsigned byte_off)
{
    return *(gptr<T>)(reinterpret_cast<char *>(base) + byte_off);
}

template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T &at(const T *base,
                                                                         unsigned byte_off)
{
    return *(gptr<const T>)(reinterpret_cast<const char *>(base) + byte_off);
}

__device__ __forceinline__ double fx_value(unsigned long long q, double jq_inv)
{
    return (double)(long long)q * jq_inv;
}

// 1/x and 1/sqrt(x): the hardware approximations (about 1 ulp) in FP32, exact
// division and square root in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt1(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt1(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ int pack_cell(int ix, int iy)
{
    return (int)((unsigned)ix | ((unsigned)iy << 16));
}
__device__ __forceinline__ int cell_x(int c) { return c & 0xffff; }

// Tiles the fold searches on each side along an axis of n cells.  A tile's
// current block spans its cells plus one guard below and two above, so the
// entries on a cell come from the tile's own block and its neighbours' --
// unless the last tile along the axis is one cell wide: the guards of the
// tile before it then reach over it into the next tile, two tiles away.
__host__ __device__ constexpr int fold_reach(int n, int size) { return n % size == 1 ? 2 : 1; }

// Offset of cell l of tile t within the block of tile t + o (periodic, n
// cells, tiles of `size` cells with a shorter last one).
__device__ __forceinline__ int span_off(int l, int o, int t, int n, int size)
{
    const int nt = (n + size - 1) / size;
    int p = l;
    if (o < 0) {
        for (int k = 1; k <= -o; ++k) {
            const int a = wrapi(t - k, nt);
            p += min(size, n - a * size);
        }
    } else {
        for (int k = 0; k < o; ++k) {
            const int a = wrapi(t + k, nt);
            p -= min(size, n - a * size);
        }
    }
    return p;
}
__device__ __forceinline__ int cell_y(int c) { return (int)((unsigned)c >> 16); }

// window coordinate of storage column gx (>= nx means the gap)
__device__ __forceinline__ int window_col(int gx, int origin, int nxs)
{
    int w = gx - origin;
    return w < 0 ? w + nxs : w;
}

// A batch of simulations stepped by shared launches: the kernels read the
// work list (simulation, tile) and a descriptor table from device memory.
struct BatchDev {
    int nwork;        // entries of the work list in use
    int nsim;         // descriptors in use
    const int2 *work; // (simulation, tile), simulations in contiguous runs
    int blocks_done;  // blocks of the running launch that finished
    // streaming field kernels (when every simulation has the same filter
    // halo): (simulation, unit) lists of the fold and of the filter + Yee
    int nfold, nyee;
    const int2 *fold_work;
    const int2 *yee_work;
};
template <typename R>
hipError_t launch_batch_step(const SimDev<R> *ds, const BatchDev *b, int grid, hipStream_t s,
                             int rf = -1, int grid_fold = 0, int grid_yee = 0);

// Launchers (defined in pic_kernels.hip for R = float and double).
// The single-simulation step folds the current inside the Yee launch when
// every tile has one float image (reduction deposit, one block per tile) and
// the filter halo is at most one cell; otherwise the fold runs as a launch of
// its own before it.  A Yee strip folds its rows plus 1 + 2 halo rows of the
// current, so a wider halo costs more re-folded rows than the separate launch
// (measured on the 2000 x 512 laser wakefield with the compensated filter).
template <typename R> inline bool folds_in_yee(const SimDev<R> &d)
{
    const int rf = d.npass > 0 ? d.npass + (d.compensate ? 1 : 0) : 0;
    return !d.direct && d.nsb == 1 && rf <= 1;
}

template <typename R> struct Launch {
    static hipError_t push_deposit(const SimDev<R> &d, hipStream_t s);
    // rewrite the push's work order, heaviest items first
    static hipError_t order(const SimDev<R> &d, hipStream_t s);
    // the particle layouts of the n simulations of a batch's descriptor table
    static hipError_t layout_b(const SimDev<R> *ds, int n, hipStream_t s);
    // only_if_shift: skip unless the last step shifted the moving window;
    // unpend = false leaves clearing the pending flag to the window launch
    static hipError_t settle(const SimDev<R> &d, hipStream_t s, bool only_if_shift = false,
                             bool unpend = true);
    static hipError_t fold(const SimDev<R> &d, int nplanes, R *o0, R *o1, R *o2, hipStream_t s);
    // before_shift (three planes only): keep the window gap of the last
    // step's deposit although that step's end has shifted the window
    static hipError_t filter(const SimDev<R> &d, int nplanes, const R *i0, const R *i1,
                             const R *i2, R *o0, R *o1, R *o2, hipStream_t s,
                             bool before_shift = false);
    // filter + Yee (+ the fold, where folds_in_yee) and the step's end
    static hipError_t yee(const SimDev<R> &d, hipStream_t s);
    static hipError_t window(const SimDev<R> &d, hipStream_t s);
    static hipError_t load(const SimDev<R> &d, int sp, hipStream_t s);
    static hipError_t rho(const SimDev<R> &d, hipStream_t s);
    static hipError_t g0(const SimDev<R> &d, hipStream_t s);
    static hipError_t diag(const SimDev<R> &d, int has_prev, hipStream_t s);
    static hipError_t copy_plane(const R *src, R *dst, long long n, hipStream_t s);
};

}  // namespace pic
