// HIP kernels for gfx950 of one 2D EM-PIC timestep (paper Sec. 2.2, Fig. 1):
// stage 1 interpolation, stage 2 Boris push, stage 3 charge-conserving
// deposit (+ filter), stage 4 Yee FDTD; plus the tile hand-off of particles
// (the paper's particle transfer between regions, Sec. 3.2) and the moving
// window and loading of Sec. 4.1.  Every kernel is a template over the working
// precision R (float for the production path, double for the FP64 path).
#include "pic_dev.h"

#include <algorithm>

namespace pic {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R lerp2(const R *f, int i, int j, R wx, R wy)
{
    // bilinear value on the corner (i, j) of an LDS tile block, i, j >= -1
    const R *p = f + (i + 1) + (j + 1) * PX;
    const R a = p[0] + wx * (p[1] - p[0]);
    const R b = p[PX] + wx * (p[PX + 1] - p[PX]);
    return a + wy * (b - a);
}

// Inclusive-exclusive block scan of a predicate: returns the exclusive rank of
// this thread's `pred` among the block and writes the block total to *total.
__device__ int block_rank(bool pred, int *s_w, int *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long m = __ballot(pred);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[wv] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < NT / 64; ++k) {
        const int c = s_w[k];
        off += (k < wv) ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return off + before;
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box with
// multipliers 0xD2511F53, 0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85.
__device__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t a = c[0], b = c[2];
        const uint32_t lo0 = 0xD2511F53u * a, hi0 = __umulhi(0xD2511F53u, a);
        const uint32_t lo1 = 0xCD9E8D57u * b, hi1 = __umulhi(0xCD9E8D57u, b);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Maxwellian momentum of the particle loaded at (lab cell x, cell y,
// sub-position) of species s: Box-Muller in double on both word pairs.
template <typename R>
__device__ void maxwellian(const SpDev<R> &P, uint32_t key0, uint32_t key1, uint32_t ilab,
                           uint32_t j, uint32_t sub, uint32_t s, R *u)
{
    uint32_t c[4] = {ilab, j, sub, s};
    philox4x32_10(c, key0, key1);
    const double two32 = 4294967296.0;
    const double r0 = sqrt(-2.0 * log(((double)c[0] + 1.0) / two32));
    const double a0 = 2.0 * M_PI * ((double)c[1] / two32);
    const double r1 = sqrt(-2.0 * log(((double)c[2] + 1.0) / two32));
    const double a1 = 2.0 * M_PI * ((double)c[3] / two32);
    const double n0 = r0 * cos(a0), n1 = r0 * sin(a0), n2 = r1 * cos(a1);
    u[0] = (R)(P.ufl[0] + P.uth[0] * n0);
    u[1] = (R)(P.ufl[1] + P.uth[1] * n1);
    u[2] = (R)(P.ufl[2] + P.uth[2] * n2);
}

// ---------------------------------------------------------------------------
// stage 3: Villasenor-Buneman deposit of one straight segment that lies in
// the cell (lx+cx, ly+cy) of the tile block (prefactors qjx, qjy, qp include
// the fixed-point scale).  The segment is the part
// t in [ta, tb] of the step of a particle starting at offset (x, y) of cell
// (lx, ly) with displacement (ddx, ddy) cells.  Its x extent is (tb-ta)*ddx,
// taken from the displacement rather than from differences of positions so
// that slow particles keep full relative accuracy in FP32.
// Jz uses the exact time average of the bilinear node weight along the
// segment: weight at the midpoint +- (extent_x * extent_y)/12.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void deposit_segment(unsigned long long *sj, int lx, int ly, R x, R y,
                                                R ddx, R ddy, R vz, R qjx, R qjy, R qp, R ta,
                                                R tb, int cx, int cy)
{
    const R f = tb - ta;
    const R tm = R(0.5) * (ta + tb);
    const R xm = x + tm * ddx - (R)cx;
    const R ym = y + tm * ddy - (R)cy;
    const R sx = f * ddx, sy = f * ddy;
    const R ax = qjx * sx, ay = qjy * sy;
    const R az = qp * vz * f, corr = sx * sy * R(1.0 / 12.0);
    const int k = (lx + cx + 1) + (ly + cy + 1) * PX;
    unsigned long long *jx = sj, *jy = sj + BP, *jz = sj + 2 * BP;
    lds_acc(jx + k, ax * (R(1) - ym));
    lds_acc(jx + k + PX, ax * ym);
    lds_acc(jy + k, ay * (R(1) - xm));
    lds_acc(jy + k + 1, ay * xm);
    lds_acc(jz + k, az * ((R(1) - xm) * (R(1) - ym) + corr));
    lds_acc(jz + k + 1, az * (xm * (R(1) - ym) - corr));
    lds_acc(jz + k + PX, az * ((R(1) - xm) * ym - corr));
    lds_acc(jz + k + PX + 1, az * (xm * ym + corr));
}

// Split the straight move at the cell boundaries it crosses (at most one per
// axis since |ddx|, |ddy| < 1), in the order the path crosses them.
template <typename R>
__device__ __forceinline__ void deposit_move(unsigned long long *sj, int lx, int ly, R x, R y,
                                             R ddx, R ddy, R vz, R qjx, R qjy, R qp)
{
    const R x1 = x + ddx, y1 = y + ddy;
    const int di = (x1 >= R(1)) - (x1 < R(0));
    const int dj = (y1 >= R(1)) - (y1 < R(0));
    R tx = R(1), ty = R(1);
    if (di) tx = fmin(((di > 0 ? R(1) : R(0)) - x) * rcp(ddx), R(1));
    if (dj) ty = fmin(((dj > 0 ? R(1) : R(0)) - y) * rcp(ddy), R(1));
    const bool xfirst = tx <= ty;
    const R t1 = xfirst ? tx : ty, t2 = xfirst ? ty : tx;
    if (t1 > R(0))
        deposit_segment(sj, lx, ly, x, y, ddx, ddy, vz, qjx, qjy, qp, R(0), t1, 0, 0);
    if (t2 > t1)
        deposit_segment(sj, lx, ly, x, y, ddx, ddy, vz, qjx, qjy, qp, t1, t2, xfirst ? di : 0,
                        xfirst ? 0 : dj);
    if (R(1) > t2)
        deposit_segment(sj, lx, ly, x, y, ddx, ddy, vz, qjx, qjy, qp, t2, R(1), di, dj);
}

// Load the six field planes of buffer `par` on the tile block (periodic wrap
// in storage; gap columns hold zeros) and clear the current block.
template <int BT, typename R>
__device__ __forceinline__ void load_tile_fields(const SimDev<R> &d, int par, int x0, int y0,
                                                 int w, int h, R *sf, unsigned long long *sj)
{
    for (int k = threadIdx.x; k < BP; k += BT) {
        const int lx = k % PX - 1, ly = k / PX - 1;
        const bool in = lx < w + 2 && ly < h + 2;
        const int gx = wrapi(x0 + lx, d.nxs), gy = wrapi(y0 + ly, d.ny);
        const size_t g = in ? (size_t)gx + (size_t)gy * d.nxs : 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const gptr<const R> Fc = glob<const R>(par ? d.F[1][c] : d.F[0][c]);
            sf[c * BP + k] = in ? Fc[g] : R(0);
        }
        if (sj) {
            sj[k] = 0ull;
            sj[BP + k] = 0ull;
            sj[2 * BP + k] = 0ull;
        }
    }
}

// Filled in by the first N_DIR threads of a block for species P: the 8
// neighbour tiles of t, the direction a leaver of each must have to come to
// t, and the exclusive prefix of their outbox lengths (outbox ob, or empty
// runs when nothing is pending).  Returns nothing; needs a barrier after.
template <typename R>
__device__ __forceinline__ void neighbour_runs(const SimDev<R> &d, const SpDev<R> &P, int t,
                                               int ob, bool pend, int *s_nb,
                                               unsigned char *s_want, int *s_len)
{
    if (threadIdx.x < N_DIR) {
        const int tx = t % d.ntx, ty = t / d.ntx;
        const int k9 = threadIdx.x < 4 ? threadIdx.x : threadIdx.x + 1;
        const int ox = k9 % 3 - 1, oy = k9 / 3 - 1;
        const int nb = wrapi(tx + ox, d.ntx) + wrapi(ty + oy, d.nty) * d.ntx;
        s_nb[threadIdx.x] = nb;
        // particles that moved from nb into t stepped by (-ox, -oy)
        s_want[threadIdx.x] = (unsigned char)dir_index(-ox, -oy);
        s_len[threadIdx.x] = pend ? glob(P.ob_count[ob])[nb] : 0;
    }
}

// ---------------------------------------------------------------------------
// rows a1-a4: the advance of one tile (the paper's region, Sec. 3.2) and
// step.  Every particle of the tile (buffer ppar) and every leaver of the
// previous push that came to this tile (outbox opar, if pending) is
// interpolated, pushed and deposited; particles that stay are written
// compacted to buffer ppar ^ 1, one contiguous run per wavefront, and the ones
// that leave go to outbox opar ^ 1 with their direction.  Particles leaving
// the moving window are dropped.
//
// A block first gathers the arrivals of each species into a list in LDS (the
// outbox slots of the neighbours' leavers whose direction points at this
// tile), then runs one stream per species over its own particles followed by
// that list, so the arrivals fill the last, partial batch of the tile's own
// particles instead of taking batches of their own.
// ---------------------------------------------------------------------------
// Entries of the arrival list per push block (all species of the block share
// it): 16 KB of LDS beside the 17 KB field and current blocks leaves room for
// four 512-thread blocks per CU; 1024-thread blocks run two per CU.
template <int BT> struct ArrivalCap { static constexpr int n = BT >= 1024 ? 12288 : 4096; };

template <typename R, int LCAP>
struct PushShared {
    R sf[6 * BP];                 // E, B of the tile block
    unsigned long long sj[3 * BP];  // Jx, Jy, Jz of the tile block (fixed point)
    int arr[LCAP];                // arrivals: outbox slot of each
    int n_arr[MAX_SP];            // arrivals found per species
    int n_out[MAX_SP];            // stayers written per species
    int n_ob[MAX_SP];             // leavers written per species
};

// Zero the per-species counters (before the barrier that precedes a tile).
template <typename R, int LCAP>
__device__ __forceinline__ void push_counters_zero(PushShared<R, LCAP> &sh)
{
    if (threadIdx.x < MAX_SP) {
        sh.n_arr[threadIdx.x] = 0;
        sh.n_out[threadIdx.x] = 0;
        sh.n_ob[threadIdx.x] = 0;
    }
}

// Append to `list` (capacity lcap; the count in *n) the outbox-ob slots of
// species P's leavers that the 8 neighbours of tile (tx, ty) sent to it.  All
// threads of the block take part; no barrier.  Every wavefront reads the 8
// outbox lengths itself (lanes 0..7) and forms their prefix with lane
// shuffles.  A leaver of neighbour k (k9 = k or k + 1, skipping the centre,
// offset (k9 % 3 - 1, k9 / 3 - 1)) came to this tile if its direction is
// dir_index of the opposite offset, which is 7 - k.
template <int BT, typename R>
__device__ __forceinline__ void gather_arrivals(const SimDev<R> &d, const SpDev<R> &P, int tx,
                                                int ty, int ob, int *list, int lcap, int *n)
{
    const int lane = threadIdx.x & 63;
    int len = 0;
    if (lane < N_DIR) {
        const int k9 = lane < 4 ? lane : lane + 1;
        const int nb = wrapi(tx + k9 % 3 - 1, d.ntx) + wrapi(ty + k9 / 3 - 1, d.nty) * d.ntx;
        len = glob(P.ob_count[ob])[nb];
    }
    int inc = len;  // inclusive prefix over lanes 0..7
#pragma unroll
    for (int o = 1; o < N_DIR; o <<= 1) {
        const int v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    int pre[N_DIR + 1];
    pre[0] = 0;
#pragma unroll
    for (int k = 0; k < N_DIR; ++k) pre[k + 1] = __builtin_amdgcn_readlane(inc, k);
    const int total = pre[N_DIR];
    const unsigned long long below = (1ull << lane) - 1ull;
    const gptr<const unsigned char> dirs = glob<const unsigned char>(P.ob_dir[ob]);
    for (int e0 = 0; e0 < total; e0 += BT) {
        const int e = e0 + (int)threadIdx.x;
        bool take = false;
        int o = 0;
        if (e < total) {
            int k = 0, start = 0;
#pragma unroll
            for (int j = 1; j < N_DIR; ++j) {
                const bool past = e >= pre[j];
                k += past ? 1 : 0;
                start = past ? pre[j] : start;
            }
            const int k9 = k < 4 ? k : k + 1;
            const int nb = wrapi(tx + k9 % 3 - 1, d.ntx) + wrapi(ty + k9 / 3 - 1, d.nty) * d.ntx;
            o = nb * d.cap_out + (e - start);
            take = dirs[o] == (unsigned char)(N_DIR - 1 - k);
        }
        const unsigned long long m = __ballot(take);
        if (m) {
            int off = 0;
            if (lane == 0) off = atomicAdd(n, (int)__popcll(m));
            off = __builtin_amdgcn_readfirstlane(off);
            const int q = off + (int)__popcll(m & below);
            if (take && q < lcap) list[q] = o;
        }
    }
}

// Steps of inflow a segment must still have room for after a push; with
// fewer free slots the push asks for a relayout at the end of the step.
// Between the periodic checks a tile's inflow can rise several-fold (dense
// bunches of a two-stream instability sweeping into it), faster than room
// reserved from the inflow seen at the last check covers.
constexpr int RELAY_STEPS = 4;

// One tile (t) of one push: g selects the species when d.nsb > 1 species
// blocks share a tile (this block then pushes species g only and leaves its
// current block as exact 64-bit sums in slice g of the tile; the fold adds
// the slices as integers before converting, so the result is the same bits as
// one block pushing every species).  Needs the counters of `sh` zeroed and a
// barrier before; ends without a barrier, with the counters zeroed again.
template <int BT, bool DIRECT, typename R, int LCAP>
__device__ __forceinline__ void push_tile(const SimDev<R> &d, const int t, const int g,
                                          const int nsb, PushShared<R, LCAP> &sh)
{
    R *const sf = sh.sf;
    unsigned long long *const sj = sh.sj;
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const gptr<const DevState> st = glob<const DevState>(d.st);
    const int par = st->parity, origin = st->origin;
    const int pp = st->ppar, ob = st->opar;
    const bool pend = st->pend != 0;
    const int s0 = nsb > 1 ? g : 0, s1 = nsb > 1 ? g + 1 : d.nsp;
    const int lcap = LCAP / max(s1 - s0, 1);
    load_tile_fields<BT>(d, par, x0, y0, w, h, sf, sj);
    if (pend)
        for (int s = s0; s < s1; ++s)
            gather_arrivals<BT>(d, d.sp[s], tx, ty, ob, sh.arr + (s - s0) * lcap, lcap,
                                &sh.n_arr[s]);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const R jq = d.jq;
    const size_t obase = (size_t)t * d.cap_out;
    for (int s = s0; s < s1; ++s) {
        const SpDev<R> &P = d.sp[s];
        const PartBuf<R> &bi = P.pb[pp];
        const PartBuf<R> &bo = P.pb[pp ^ 1];
        const unsigned n_own = (unsigned)glob(bi.count)[t];
        const int n_found = sh.n_arr[s];
        const unsigned n_tot = n_own + (unsigned)min(n_found, lcap);
        const int *const list = sh.arr + (s - s0) * lcap;
        // the tile's segments: input at buffer ppar's layout, output at
        // buffer ppar ^ 1's (a relayout changes only the latter)
        const size_t base = seg_start(P, pp, t), obase_p = seg_start(P, pp ^ 1, t);
        const int ocap = seg_slots(P, pp ^ 1, t);
        // tile-uniform base pointers, indexed with 32-bit offsets
        const int *const ic = bi.cell + base;
        const R *const ixp = bi.x + base;
        const R *const iyp = bi.y + base;
        const R *const iux = bi.ux + base;
        const R *const iuy = bi.uy + base;
        const R *const iuz = bi.uz + base;
        int *const oc = bo.cell + obase_p;
        R *const oxp = bo.x + obase_p;
        R *const oyp = bo.y + obase_p;
        R *const oux = bo.ux + obase_p;
        R *const ouy = bo.uy + obase_p;
        R *const ouz = bo.uz + obase_p;
        // deposit prefactors carry the fixed-point scale (a power of two)
        const R qjx = P.qp * d.jxs * jq, qjy = P.qp * d.jys * jq, qps = P.qp * jq;
        const R tau = P.tau;
        // Push, move and deposit one particle per lane (act: the lane holds
        // one), then write the wavefront's stayers and leavers.
        auto advance = [&](bool act, int cell, R x, R y, R ux, R uy, R uz) {
            bool stay = false, send = false;
            int ncell = 0, dir = 0;
            R xn = 0, yn = 0;
            if (act) {
                const int ix = cell_x(cell), iy = cell_y(cell);
                const int lx = ix - x0, ly = iy - y0;
                // stage 1: each component from its own staggered grid
                const bool lox = x < R(0.5), loy = y < R(0.5);
                const int ixh = lx - (lox ? 1 : 0), iyh = ly - (loy ? 1 : 0);
                const R wxh = x + (lox ? R(0.5) : R(-0.5));
                const R wyh = y + (loy ? R(0.5) : R(-0.5));
                const R ex = lerp2(sf, ixh, ly, wxh, y);
                const R ey = lerp2(sf + BP, lx, iyh, x, wyh);
                const R ez = lerp2(sf + 2 * BP, lx, ly, x, y);
                const R bx = lerp2(sf + 3 * BP, lx, iyh, x, wyh);
                const R by = lerp2(sf + 4 * BP, ixh, ly, wxh, y);
                const R bz = lerp2(sf + 5 * BP, ixh, iyh, wxh, wyh);
                // stage 2: relativistic Boris
                const R umx = ux + tau * ex, umy = uy + tau * ey, umz = uz + tau * ez;
                const R ig = rsqrt1(R(1) + umx * umx + umy * umy + umz * umz);
                const R tvx = tau * bx * ig, tvy = tau * by * ig, tvz = tau * bz * ig;
                const R upx = umx + (umy * tvz - umz * tvy);
                const R upy = umy + (umz * tvx - umx * tvz);
                const R upz = umz + (umx * tvy - umy * tvx);
                const R fs = R(2) * rcp(R(1) + tvx * tvx + tvy * tvy + tvz * tvz);
                const R svx = fs * tvx, svy = fs * tvy, svz = fs * tvz;
                ux = umx + (upy * svz - upz * svy) + tau * ex;
                uy = umy + (upz * svx - upx * svz) + tau * ey;
                uz = umz + (upx * svy - upy * svx) + tau * ez;
                // move and stage 3
                const R ig2 = rsqrt1(R(1) + ux * ux + uy * uy + uz * uz);
                const R ddx = d.dt_dx * ux * ig2, ddy = d.dt_dy * uy * ig2;
                deposit_move(sj, lx, ly, x, y, ddx, ddy, uz * ig2, qjx, qjy, qps);
                xn = x + ddx;
                yn = y + ddy;
                int di = (xn >= R(1)) - (xn < R(0));
                int dj = (yn >= R(1)) - (yn < R(0));
                xn -= (R)di;
                yn -= (R)dj;
                // x + ddx in (-2^-25, 0) rounds to exactly 1 after adding 1
                if (xn >= R(1)) { xn -= R(1); di += 1; }
                if (yn >= R(1)) { yn -= R(1); dj += 1; }
                const int nix = wrapi(ix + di, d.nxs), niy = wrapi(iy + dj, d.ny);
                const bool dead = d.window && window_col(nix, origin, d.nxs) >= d.nx;
                // tile step; a tile that is the whole period wraps onto itself
                const int dtx = d.ntx == 1 ? 0 : (lx + di >= w ? 1 : (lx + di < 0 ? -1 : 0));
                const int dty = d.nty == 1 ? 0 : (ly + dj >= h ? 1 : (ly + dj < 0 ? -1 : 0));
                ncell = pack_cell(nix, niy);
                send = !dead && (dtx || dty);
                stay = !dead && !send;
                dir = dir_index(dtx, dty);
            }
            // stayers: one contiguous run per wavefront in buffer ppar ^ 1
            // (every lane of the wavefront runs this part: lane 0 is active
            // and readfirstlane gives its value to the others)
            const unsigned long long ms = __ballot(stay);
            if (ms) {
                int off = 0;
                if (lane == 0) off = atomicAdd(&sh.n_out[s], (int)__popcll(ms));
                off = __builtin_amdgcn_readfirstlane(off);
                if (stay) {
                    const unsigned q = (unsigned)(off + (int)__popcll(ms & below));
                    if (q < (unsigned)ocap) {
                        const unsigned o4 = q * 4u, oR = q * (unsigned)sizeof(R);
                        at(oc, o4) = ncell;
                        at(oxp, oR) = xn;
                        at(oyp, oR) = yn;
                        at(oux, oR) = ux;
                        at(ouy, oR) = uy;
                        at(ouz, oR) = uz;
                    } else {
                        __hip_atomic_fetch_or(&glob(d.st)->err, ERR_SEG, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            // leavers: one contiguous run per wavefront in outbox opar ^ 1
            const unsigned long long ml = __ballot(send);
            if (ml) {
                int off = 0;
                if (lane == 0) off = atomicAdd(&sh.n_ob[s], (int)__popcll(ml));
                off = __builtin_amdgcn_readfirstlane(off);
                if (send) {
                    const int slot = off + (int)__popcll(ml & below);
                    if (slot < d.cap_out) {
                        const size_t o = obase + slot;
                        glob(P.ob_cell[ob ^ 1])[o] = ncell;
                        glob(P.ob_dir[ob ^ 1])[o] = (unsigned char)dir;
                        glob(P.ob_x[ob ^ 1])[o] = xn;
                        glob(P.ob_y[ob ^ 1])[o] = yn;
                        glob(P.ob_ux[ob ^ 1])[o] = ux;
                        glob(P.ob_uy[ob ^ 1])[o] = uy;
                        glob(P.ob_uz[ob ^ 1])[o] = uz;
                    } else {
                        __hip_atomic_fetch_or(&glob(d.st)->err, ERR_OUTBOX, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        };
        // Particle i of the stream: own particle i, or arrival i - n_own.
        auto fetch = [&](unsigned i, int &c, R &x, R &y, R &ux, R &uy, R &uz) {
            if (i < n_own) {
                const unsigned o4 = i * 4u, oR = i * (unsigned)sizeof(R);
                c = at(ic, o4);
                x = at(ixp, oR);
                y = at(iyp, oR);
                ux = at(iux, oR);
                uy = at(iuy, oR);
                uz = at(iuz, oR);
            } else if (i < n_tot) {
                const size_t o = (size_t)list[i - n_own];
                c = glob(P.ob_cell[ob])[o];
                x = glob(P.ob_x[ob])[o];
                y = glob(P.ob_y[ob])[o];
                ux = glob(P.ob_ux[ob])[o];
                uy = glob(P.ob_uy[ob])[o];
                uz = glob(P.ob_uz[ob])[o];
            }
        };
        // The stream, read one batch ahead: the loads of batch k+1 are in
        // flight while batch k is pushed and deposited.
        int nc = 0;
        R nxv = 0, nyv = 0, nux = 0, nuy = 0, nuz = 0;
        fetch(threadIdx.x, nc, nxv, nyv, nux, nuy, nuz);
        for (unsigned p0 = 0; p0 < n_tot; p0 += BT) {
            const unsigned p = p0 + threadIdx.x;
            const int cell = nc;
            const R x = nxv, y = nyv, ux = nux, uy = nuy, uz = nuz;
            fetch(p + BT, nc, nxv, nyv, nux, nuy, nuz);
            advance(p < n_tot, cell, x, y, ux, uy, uz);
        }
        if (threadIdx.x == 0 && n_found > lcap)
            __hip_atomic_fetch_or(&glob(d.st)->err, ERR_ARRIVALS, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // counts of the tile, the input buffer's segment set to the output's
    // layout (so both buffers share it after a relayout; no other block reads
    // this tile's entries), and the counters zeroed for the block's next tile
    if ((int)threadIdx.x < s1 - s0) {
        const int s = s0 + (int)threadIdx.x;
        const SpDev<R> &P = d.sp[s];
        const int ocap = seg_slots(P, pp ^ 1, t);
        const int kept = min(sh.n_out[s], ocap);
        // fewer free slots than RELAY_STEPS more steps of this step's
        // inflow: the step end lays the segments out anew (a plain store of
        // 1, so any block may make it)
        if (kept + RELAY_STEPS * sh.n_arr[s] + 64 > ocap) glob(d.st)->relay = 1;
        glob(P.pb[pp ^ 1].count)[t] = kept;
        glob(P.ob_count[ob ^ 1])[t] = min(sh.n_ob[s], d.cap_out);
        glob(P.start[pp])[t] = glob(P.start[pp ^ 1])[t];
        glob(P.seg[pp])[t] = ocap;
        if (pend) glob(P.inflow)[t] = sh.n_arr[s];  // what entered the tile this step
        sh.n_arr[s] = 0;
        sh.n_out[s] = 0;
        sh.n_ob[s] = 0;
    }

    // one flush of the tile's current block per step
    const double jqi = d.jq_inv;
    if (DIRECT) {
        // add the block into J: no other tile of this launch's colour touches
        // these cells (same-colour tiles are two tiles apart)
        for (int k = threadIdx.x; k < 3 * BP; k += BT) {
            const int c = k / BP, kk = k - c * BP;
            const int lx = kk % PX - 1, ly = kk / PX - 1;
            if (lx >= w + 2 || ly >= h + 2) continue;  // beyond a ragged tile's guards
            const size_t gi = (size_t)wrapi(x0 + lx, d.nxs) + (size_t)wrapi(y0 + ly, d.ny) * d.nxs;
            const gptr<R> J = glob(d.J[c]);
            J[gi] = J[gi] + (R)fx_value(sj[k], jqi);
        }
    } else if (nsb > 1) {
        const gptr<unsigned long long> out = glob(
            reinterpret_cast<unsigned long long *>(d.blk) + ((size_t)t * nsb + g) * 3 * BP);
        for (int k = threadIdx.x; k < 3 * BP; k += BT) out[k] = sj[k];
    } else {
        const gptr<R> out = glob(d.blk + (size_t)t * 3 * BP);
        for (int k = threadIdx.x; k < 3 * BP; k += BT) out[k] = (R)fx_value(sj[k], jqi);
    }
}

// One tile per block (batched and colour-phased launches).
template <int BT, bool DIRECT, typename R>
__device__ __forceinline__ void push_body(const SimDev<R> &d, const int t)
{
    __shared__ PushShared<R, ArrivalCap<BT>::n> sh;
    push_counters_zero(sh);
    __syncthreads();
    push_tile<BT, DIRECT>(d, t, 0, 1, sh);
}

// After each push: both buffers flip and its outbox is pending.
template <typename R>
__device__ __forceinline__ void push_end_body(const SimDev<R> &d)
{
    DevState *st = d.st;
    st->ppar ^= 1;
    st->opar ^= 1;
    st->pend = 1;
}

// Append the pending leavers (outbox opar) to the tiles they moved into, so
// that buffer ppar holds every particle.  One wavefront per tile; ranks from
// ballots, so the order is deterministic.  k_unpend then clears the flag.
constexpr int MT = 64;

template <typename R>
__global__ __launch_bounds__(MT) void k_settle(SimDev<R> d, int only_if_shift)
{
    __shared__ int s_nb[N_DIR], s_len[N_DIR];
    __shared__ unsigned char s_want[N_DIR];
    const DevState *st = d.st;
    if (only_if_shift && !st->shift) return;
    if (!st->pend) return;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int pp = st->ppar, ob = st->opar;
    const int lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int s = 0; s < d.nsp; ++s) {
        const SpDev<R> &P = d.sp[s];
        neighbour_runs(d, P, t, ob, true, s_nb, s_want, s_len);
        __syncthreads();
        int pre[N_DIR + 1];
        pre[0] = 0;
        for (int k = 0; k < N_DIR; ++k) pre[k + 1] = pre[k] + s_len[k];
        const PartBuf<R> &B = P.pb[pp];
        const int n0 = B.count[t];
        const size_t base = seg_start(P, pp, t);
        const int cap = seg_slots(P, pp, t);
        int added = 0;
        for (int e0 = 0; e0 < pre[N_DIR]; e0 += MT) {
            const int e = e0 + lane;
            bool take = false;
            size_t o = 0;
            if (e < pre[N_DIR]) {
                int k = 0;
                while (k < N_DIR - 1 && e >= pre[k + 1]) ++k;
                o = (size_t)s_nb[k] * d.cap_out + (e - pre[k]);
                take = P.ob_dir[ob][o] == s_want[k];
            }
            const unsigned long long m = __ballot(take);
            if (take) {
                const int q = n0 + added + (int)__popcll(m & below);
                if (q < cap) {
                    const size_t dst = base + q;
                    B.cell[dst] = P.ob_cell[ob][o];
                    B.x[dst] = P.ob_x[ob][o];
                    B.y[dst] = P.ob_y[ob][o];
                    B.ux[dst] = P.ob_ux[ob][o];
                    B.uy[dst] = P.ob_uy[ob][o];
                    B.uz[dst] = P.ob_uz[ob][o];
                } else {
                    atomicOr(&d.st->err, ERR_SETTLE);
                }
            }
            added += (int)__popcll(m);
        }
        if (lane == 0) {
            B.count[t] = min(n0 + added, cap);
            glob(P.inflow)[t] = added;  // what entered the tile this step
        }
        __syncthreads();
    }
}

template <typename R>
__global__ void k_unpend(SimDev<R> d, int only_if_shift)
{
    if (threadIdx.x == 0 && !(only_if_shift && !d.st->shift)) d.st->pend = 0;
}

// ---------------------------------------------------------------------------
// row a5: fold the per-tile blocks into the global planes.  Each cell sums, in
// a fixed order, the block entries of the (up to 9) tile images whose block
// covers it; gap columns of the moving window are cleared (current deposited
// beyond the window is dropped).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void fold_body(const SimDev<R> &d, const int t, int nplanes, R *o0,
                                          R *o1, R *o2)
{
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const int origin = glob(d.st)->origin;
    for (int k = threadIdx.x; k < w * h; k += NT) {
        const int lx = k % w, ly = k / w;
        const int gx = x0 + lx, gy = y0 + ly;
        R a0 = 0, a1 = 0, a2 = 0;
        for (int oy = -d.ry; oy <= d.ry; ++oy) {
            const int tyn = wrapi(ty + oy, d.nty);
            const int hn = min(TY, d.ny - tyn * TY);
            const int py = span_off(ly, oy, ty, d.ny, TY);
            if (py < -1 || py >= hn + 2) continue;
            for (int ox = -d.rx; ox <= d.rx; ++ox) {
                const int txn = wrapi(tx + ox, d.ntx);
                const int wn = min(TX, d.nxs - txn * TX);
                const int px = span_off(lx, ox, tx, d.nxs, TX);
                if (px < -1 || px >= wn + 2) continue;
                const gptr<const R> b = glob<const R>(
                    d.blk + (size_t)(txn + tyn * d.ntx) * 3 * BP + (px + 1) + (py + 1) * PX);
                a0 += b[0];
                if (nplanes > 1) {
                    a1 += b[BP];
                    a2 += b[2 * BP];
                }
            }
        }
        const bool gap = d.window && window_col(gx, origin, d.nxs) >= d.nx;
        const size_t g = (size_t)gx + (size_t)gy * d.nxs;
        glob(o0)[g] = gap ? R(0) : a0;
        if (nplanes > 1) {
            glob(o1)[g] = gap ? R(0) : a1;
            glob(o2)[g] = gap ? R(0) : a2;
        }
    }
}

// ---------------------------------------------------------------------------
// row a6: binomial filter.  Per tile: load the planes with a halo of
// rf = npass + compensate cells, apply the x passes (binomial, then
// compensator), then the y passes, keeping the gap at zero; write the
// interior.  All planes go through each pass together.  A pass only touches
// the rows of the halo'd tile, the x passes its halo'd columns and the y
// passes the tile's own.  Cells next to that region are never written, so
// the region's rim takes arbitrary values, but after rf passes these have
// moved at most rf - 1 cells inwards and never reach the interior.
// ---------------------------------------------------------------------------
constexpr int QB = QX * QY; // cells of one plane's filter block

template <typename R>
__device__ __forceinline__ void filter_body(const SimDev<R> &d, const int t, int nplanes,
                                            const R *i0, const R *i1, const R *i2, R *o0,
                                            R *o1, R *o2)
{
    // no contraction into fma: the tile and streaming forms (and the batched
    // launches) must round every term alike
#pragma clang fp contract(off)
    __shared__ R sa[3 * QB];
    __shared__ R sb[3 * QB];
    __shared__ unsigned char s_gap[QX];
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const int origin = glob(d.st)->origin;
    const int rf = d.npass + (d.compensate ? 1 : 0);
    const R N = (R)d.npass;
    // a single plane (the charge) also runs through the other two slots, on
    // a copy of itself, so that every loop below has a fixed trip count
    const gptr<const R> in[3] = {glob(i0), glob(nplanes > 1 ? i1 : i0),
                                 glob(nplanes > 2 ? i2 : i0)};
    for (int k = threadIdx.x; k < QX; k += NT) {
        int gx = (x0 + k - MAX_FR) % d.nxs;
        gx += gx < 0 ? d.nxs : 0;
        s_gap[k] = d.window && window_col(gx, origin, d.nxs) >= d.nx;
    }
    // rows [MAX_FR - rf, MAX_FR + h + rf) of the block hold the halo'd tile;
    // its columns are [MAX_FR - rf, MAX_FR + w + rf)
    const int k0 = (MAX_FR - rf) * QX, k1 = (MAX_FR + h + rf) * QX;
    const int ilo = MAX_FR - rf, ihi = MAX_FR + w + rf;
    // all loads go out before the first LDS store; a cell outside the
    // halo'd tile reads cell 0 and is not stored
    constexpr int FRN = (QB + NT - 1) / NT;
    R v[FRN][3];
    bool live[FRN];
#pragma unroll
    for (int r = 0; r < FRN; ++r) {
        const int k = k0 + threadIdx.x + r * NT;
        const int i = k % QX, j = k / QX;
        live[r] = k < k1 && i >= ilo && i < ihi;
        // the halo may reach beyond one period on tiny grids
        int gx = (x0 + i - MAX_FR) % d.nxs;
        gx += gx < 0 ? d.nxs : 0;
        int gy = (y0 + j - MAX_FR) % d.ny;
        gy += gy < 0 ? d.ny : 0;
        const size_t g = live[r] ? (size_t)gx + (size_t)gy * d.nxs : 0;
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) v[r][pl] = in[pl][g];
    }
#pragma unroll
    for (int r = 0; r < FRN; ++r) {
        const int k = k0 + threadIdx.x + r * NT;
        if (live[r]) {
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) sa[pl * QB + k] = v[r][pl];
        }
    }
    __syncthreads();
    R *a = sa, *b = sb;
    for (int pass = 0; pass < rf; ++pass) {
        const bool comp = pass == d.npass;
        const R w0 = comp ? -N / R(4) : R(0.25), w1 = comp ? (R(4) + R(2) * N) / R(4) : R(0.5);
        for (int k = k0 + threadIdx.x; k < k1; k += NT) {
            const int i = k % QX;
            if (i < ilo || i >= ihi) continue;
            const bool live = i > 0 && i < QX - 1 && !s_gap[i];
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const int q = pl * QB + k;
                b[q] = live ? w0 * a[q - 1] + w1 * a[q] + w0 * a[q + 1] : R(0);
            }
        }
        __syncthreads();
        R *tmp = a;
        a = b;
        b = tmp;
    }
    for (int pass = 0; pass < rf; ++pass) {
        const bool comp = pass == d.npass;
        const R w0 = comp ? -N / R(4) : R(0.25), w1 = comp ? (R(4) + R(2) * N) / R(4) : R(0.5);
        for (int k = k0 + threadIdx.x; k < k1; k += NT) {
            const int i = k % QX, j = k / QX;
            if (i < MAX_FR || i >= MAX_FR + w) continue;
            const bool live = j > 0 && j < QY - 1;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const int q = pl * QB + k;
                b[q] = live ? w0 * a[q - QX] + w1 * a[q] + w0 * a[q + QX] : R(0);
            }
        }
        __syncthreads();
        R *tmp = a;
        a = b;
        b = tmp;
    }
    R *const out[3] = {o0, o1, o2};
    for (int k = threadIdx.x; k < w * h; k += NT) {
        const int lx = k % w, ly = k / w;
        const size_t g = (size_t)(x0 + lx) + (size_t)(y0 + ly) * d.nxs;
        const int q = (lx + MAX_FR) + (ly + MAX_FR) * QX;
        for (int pl = 0; pl < nplanes; ++pl) glob(out[pl])[g] = a[pl * QB + q];
    }
}

// ---------------------------------------------------------------------------
// row a7: Yee step B half, E full, B half on a tile with its guard halo; reads
// buffer `parity`, writes the other one.  Beyond the moving window every
// component is held at zero after each sub-step, as zero guard cells would.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void yee_body(const SimDev<R> &d, const int t)
{
    // no contraction into fma: the tile and streaming forms (and the batched
    // launches) must round every term alike
#pragma clang fp contract(off)
    __shared__ R e[3 * BP];
    __shared__ R b[3 * BP];
    __shared__ R jl[3 * BP];
    __shared__ unsigned char s_gap[PX];
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const int par = glob(d.st)->parity, origin = glob(d.st)->origin;
    for (int k = threadIdx.x; k < PX; k += NT)
        s_gap[k] = d.window && window_col(wrapi(x0 + k - 1, d.nxs), origin, d.nxs) >= d.nx;
    for (int k = threadIdx.x; k < BP; k += NT) {
        const int lx = k % PX - 1, ly = k / PX - 1;
        const bool in = lx < w + 2 && ly < h + 2;
        const size_t g =
            in ? (size_t)wrapi(x0 + lx, d.nxs) + (size_t)wrapi(y0 + ly, d.ny) * d.nxs : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const gptr<const R> Fe = glob<const R>(par ? d.F[1][c] : d.F[0][c]);
            const gptr<const R> Fb = glob<const R>(par ? d.F[1][3 + c] : d.F[0][3 + c]);
            e[c * BP + k] = in ? Fe[g] : R(0);
            b[c * BP + k] = in ? Fb[g] : R(0);
            jl[c * BP + k] = in ? glob<const R>(d.Jf[c])[g] : R(0);
        }
    }
    __syncthreads();
    const R hdt = R(0.5) * d.dt;
    // B half step on local [-1, w] x [-1, h]
    for (int k = threadIdx.x; k < BP; k += NT) {
        const int i = k % PX - 1, j = k / PX - 1;
        if (i <= w && j <= h) {
            const bool gp = s_gap[i + 1];
            const R dEz_dy = (e[2 * BP + k + PX] - e[2 * BP + k]) * d.idy;
            const R dEz_dx = (e[2 * BP + k + 1] - e[2 * BP + k]) * d.idx;
            const R dEy_dx = (e[BP + k + 1] - e[BP + k]) * d.idx;
            const R dEx_dy = (e[k + PX] - e[k]) * d.idy;
            b[k] = gp ? R(0) : b[k] - hdt * dEz_dy;
            b[BP + k] = gp ? R(0) : b[BP + k] + hdt * dEz_dx;
            b[2 * BP + k] = gp ? R(0) : b[2 * BP + k] - hdt * (dEy_dx - dEx_dy);
        }
    }
    __syncthreads();
    // E full step on local [0, w] x [0, h]
    for (int k = threadIdx.x; k < BP; k += NT) {
        const int i = k % PX - 1, j = k / PX - 1;
        if (i >= 0 && j >= 0 && i <= w && j <= h) {
            const bool gp = s_gap[i + 1];
            const R dBz_dy = (b[2 * BP + k] - b[2 * BP + k - PX]) * d.idy;
            const R dBz_dx = (b[2 * BP + k] - b[2 * BP + k - 1]) * d.idx;
            const R dBy_dx = (b[BP + k] - b[BP + k - 1]) * d.idx;
            const R dBx_dy = (b[k] - b[k - PX]) * d.idy;
            e[k] = gp ? R(0) : e[k] + d.dt * (dBz_dy - jl[k]);
            e[BP + k] = gp ? R(0) : e[BP + k] + d.dt * (-dBz_dx - jl[BP + k]);
            e[2 * BP + k] = gp ? R(0) : e[2 * BP + k] + d.dt * (dBy_dx - dBx_dy - jl[2 * BP + k]);
        }
    }
    __syncthreads();
    // B half step on the interior, and write out
    const int npar = par ^ 1;
    for (int k = threadIdx.x; k < BP; k += NT) {
        const int i = k % PX - 1, j = k / PX - 1;
        if (i >= 0 && j >= 0 && i < w && j < h) {
            const bool gp = s_gap[i + 1];
            const R dEz_dy = (e[2 * BP + k + PX] - e[2 * BP + k]) * d.idy;
            const R dEz_dx = (e[2 * BP + k + 1] - e[2 * BP + k]) * d.idx;
            const R dEy_dx = (e[BP + k + 1] - e[BP + k]) * d.idx;
            const R dEx_dy = (e[k + PX] - e[k]) * d.idy;
            const R nbx = gp ? R(0) : b[k] - hdt * dEz_dy;
            const R nby = gp ? R(0) : b[BP + k] + hdt * dEz_dx;
            const R nbz = gp ? R(0) : b[2 * BP + k] - hdt * (dEy_dx - dEx_dy);
            const size_t g = (size_t)(x0 + i) + (size_t)(y0 + j) * d.nxs;
            glob(npar ? d.F[1][0] : d.F[0][0])[g] = e[k];
            glob(npar ? d.F[1][1] : d.F[0][1])[g] = e[BP + k];
            glob(npar ? d.F[1][2] : d.F[0][2])[g] = e[2 * BP + k];
            glob(npar ? d.F[1][3] : d.F[0][3])[g] = nbx;
            glob(npar ? d.F[1][4] : d.F[0][4])[g] = nby;
            glob(npar ? d.F[1][5] : d.F[0][5])[g] = nbz;
        }
    }
}

// Row a5 in streaming form, for the three current planes of one simulation:
// each wavefront folds half (FH rows) of a tile row of four horizontally
// adjacent tiles, lane L holding column L % 16 of tile 4 c + L / 16.
// Each cell adds, in ascending (oy, ox) order, the entries of the tile images
// whose block covers it, as fold_body does, so the sums agree bit for bit.
// For a full-height tile at least 3 columns wide a lane reads at most one
// image beyond its own in each direction (the left one for lx < 2, the right
// one for lx = w - 1; the lower one for rows 0 and 1, the upper one for row
// 15): all of the wavefront's loads go out first, unconditionally (a lane
// that needs no neighbour reads its own entry again and adds zero), then the
// sums.  Other tiles take the general per-cell path.
template <typename R, int NSB>
__device__ __forceinline__ void fold_s_body(const SimDev<R> &d, const int blk, R *o0, R *o1,
                                            R *o2)
{
    const int ngx = (d.ntx + 3) / 4;
    // rows FH * half .. of tile row ty
    const int rg = blk / ngx, ty = rg >> 1, half = rg & 1;
    const int tx = (blk % ngx) * 4 + (int)(threadIdx.x >> 4);
    const int lx = threadIdx.x & 15;
    if (tx >= d.ntx) return;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const int ly0 = half * FH, ly1 = min(h, ly0 + FH);
    if (lx >= w || ly0 >= ly1) return;
    const bool gap = d.window && window_col(x0 + lx, glob(d.st)->origin, d.nxs) >= d.nx;
    R *const out[3] = {o0, o1, o2};
    // entry `off` of the image of tile (a, b): a float block, or NSB > 1
    // slices of exact 64-bit sums added before the one conversion
    auto img = [&](int a, int b) { return (size_t)(a + b * d.ntx); };
    auto ent = [&](size_t tile, int off) -> R {
        if (NSB == 1) return glob<const R>(d.blk)[tile * 3 * BP + off];
        const gptr<const unsigned long long> q =
            glob(reinterpret_cast<const unsigned long long *>(d.blk)) + tile * NSB * 3 * BP + off;
        unsigned long long sum = 0;
#pragma unroll
        for (int g = 0; g < NSB; ++g) sum += q[(size_t)g * 3 * BP];
        return (R)fx_value(sum, d.jq_inv);
    };
    if (d.rx == 1 && d.ry == 1 && h == TY && w >= 3) {
        const int txl = wrapi(tx - 1, d.ntx), txr = wrapi(tx + 1, d.ntx);
        const int tyl = wrapi(ty - 1, d.nty), tyu = wrapi(ty + 1, d.nty);
        const int wl = min(TX, d.nxs - txl * TX), hl = min(TY, d.ny - tyl * TY);
        const int xo = lx < 2 ? -1 : (lx == w - 1 ? 1 : 0);
        const int txn = xo < 0 ? txl : (xo > 0 ? txr : tx);
        // column (px + 1) of the cell in its own image and in the x neighbour's
        const int cxo = lx + 1, cxn = xo < 0 ? lx + wl + 1 : (xo > 0 ? 0 : lx + 1);
        const size_t io = img(tx, ty), ixn = img(txn, ty);
        const size_t il = img(tx, tyl), ilx = img(txn, tyl);
        const size_t iu = img(tx, tyu), iux = img(txn, tyu);
        R own[FH][3], xn[FH][3], lo[2][3], lox[2][3], up[3], upx[3];
#pragma unroll
        for (int r = 0; r < FH; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                own[r][c] = ent(io, c * BP + cxo + (ly0 + r + 1) * PX);
                xn[r][c] = ent(ixn, c * BP + cxn + (ly0 + r + 1) * PX);
            }
        }
        // the lower image reaches rows 0 and 1, the upper one row 15
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo[r][c] = half ? R(0) : ent(il, c * BP + cxo + (r + hl + 1) * PX);
                lox[r][c] = half ? R(0) : ent(ilx, c * BP + cxn + (r + hl + 1) * PX);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            up[c] = half ? ent(iu, c * BP + cxo) : R(0);
            upx[c] = half ? ent(iux, c * BP + cxn) : R(0);
        }
        // one level of images: the x neighbour first when it lies to the left
        auto level = [&](R &a, R o, R n) {
            a += xo < 0 ? n : o;
            a += xo < 0 ? o : (xo > 0 ? n : R(0));
        };
#pragma unroll
        for (int r = 0; r < FH; ++r) {
            const int ly = ly0 + r;
            const size_t g = (size_t)(x0 + lx) + (size_t)(y0 + ly) * d.nxs;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                R a = 0;
                if (!half && r < 2) level(a, lo[r][c], lox[r][c]);
                level(a, own[r][c], xn[r][c]);
                if (half && r == FH - 1) level(a, up[c], upx[c]);
                glob(out[c])[g] = gap ? R(0) : a;
            }
        }
        return;
    }
    for (int ly = ly0; ly < ly1; ++ly) {
        R a[3] = {0, 0, 0};
        for (int oy = -d.ry; oy <= d.ry; ++oy) {
            const int tyn = wrapi(ty + oy, d.nty);
            const int hn = min(TY, d.ny - tyn * TY);
            const int py = span_off(ly, oy, ty, d.ny, TY);
            if (py < -1 || py >= hn + 2) continue;
            for (int ox = -d.rx; ox <= d.rx; ++ox) {
                const int txn = wrapi(tx + ox, d.ntx);
                const int wn = min(TX, d.nxs - txn * TX);
                const int px = span_off(lx, ox, tx, d.nxs, TX);
                if (px < -1 || px >= wn + 2) continue;
                const size_t b = img(txn, tyn);
#pragma unroll
                for (int c = 0; c < 3; ++c) a[c] += ent(b, c * BP + (px + 1) + (py + 1) * PX);
            }
        }
        const size_t g = (size_t)(x0 + lx) + (size_t)(y0 + ly) * d.nxs;
#pragma unroll
        for (int c = 0; c < 3; ++c) glob(out[c])[g] = gap ? R(0) : a[c];
    }
}

template <typename R, int NSB>
__global__ __launch_bounds__(64) void k_fold_s(SimDev<R> d, R *o0, R *o1, R *o2)
{
    fold_s_body<R, NSB>(d, xcd_remap(blockIdx.x, gridDim.x), o0, o1, o2);
}

// the same over a batch: work list entries (simulation, unit)
template <typename R>
__global__ __launch_bounds__(64) void k_fold_sb(const SimDev<R> *__restrict__ ds,
                                                const BatchDev *__restrict__ b)
{
    const int n = __builtin_amdgcn_readfirstlane(b->nfold);
    if ((int)blockIdx.x >= n) return;
    const int2 w = b->fold_work[xcd_remap(blockIdx.x, n)];
    const SimDev<R> &d = ds[__builtin_amdgcn_readfirstlane(w.x)];
    // batches step every simulation with one block per tile (nsb = 1)
    fold_s_body<R, 1>(d, __builtin_amdgcn_readfirstlane(w.y), d.J[0], d.J[1], d.J[2]);
}

// Row a5 for a single cell (gx, gy) of the three current planes, from the
// float tile images: the same images added in the same order as
// fold_s_body (its fast path for a full-height tile at least 3 columns wide,
// its general path otherwise), so the sums agree bit for bit.  The caller
// clears gap columns.
template <typename R>
__device__ __forceinline__ void fold_cell(const SimDev<R> &d, int gx, int gy, R (&a)[3])
{
    const int tx = gx / TX, ty = gy / TY;
    const int x0 = tx * TX, y0 = ty * TY;
    const int lx = gx - x0, ly = gy - y0;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const gptr<const R> blk = glob<const R>(d.blk);
    auto img = [&](int ia, int ib) { return (size_t)(ia + ib * d.ntx) * 3 * BP; };
    a[0] = a[1] = a[2] = R(0);
    if (d.rx == 1 && d.ry == 1 && h == TY && w >= 3) {
        const int txl = wrapi(tx - 1, d.ntx), txr = wrapi(tx + 1, d.ntx);
        const int wl = min(TX, d.nxs - txl * TX);
        const int xo = lx < 2 ? -1 : (lx == w - 1 ? 1 : 0);
        const int txn = xo < 0 ? txl : (xo > 0 ? txr : tx);
        const int cxo = lx + 1, cxn = xo < 0 ? lx + wl + 1 : (xo > 0 ? 0 : lx + 1);
        // one level of images: the x neighbour first when it lies to the left
        auto level = [&](int tyn, int row) {
            const size_t io = img(tx, tyn) + cxo + row * PX, in = img(txn, tyn) + cxn + row * PX;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // lanes without an x neighbour skip its load
                const R o = blk[io + c * BP], n = xo != 0 ? blk[in + c * BP] : R(0);
                a[c] += xo < 0 ? n : o;
                a[c] += xo < 0 ? o : (xo > 0 ? n : R(0));
            }
        };
        // the lower image reaches rows 0 and 1, the upper one row 15
        if (ly < 2) {
            const int tyl = wrapi(ty - 1, d.nty);
            level(tyl, ly + min(TY, d.ny - tyl * TY) + 1);
        }
        level(ty, ly + 1);
        if (ly == TY - 1) level(wrapi(ty + 1, d.nty), 0);
        return;
    }
    for (int oy = -d.ry; oy <= d.ry; ++oy) {
        const int tyn = wrapi(ty + oy, d.nty);
        const int hn = min(TY, d.ny - tyn * TY);
        const int py = span_off(ly, oy, ty, d.ny, TY);
        if (py < -1 || py >= hn + 2) continue;
        for (int ox = -d.rx; ox <= d.rx; ++ox) {
            const int txn = wrapi(tx + ox, d.ntx);
            const int wn = min(TX, d.nxs - txn * TX);
            const int px = span_off(lx, ox, tx, d.nxs, TX);
            if (px < -1 || px >= wn + 2) continue;
            const size_t b = img(txn, tyn) + (px + 1) + (py + 1) * PX;
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] += blk[b + c * BP];
        }
    }
}

// Row a6 in streaming form, for the three current planes of one simulation
// (the step runs the filter inside its Yee launch, k_fold_yee_s or k_yee_s;
// this kernel serves requests for the filtered current): each wavefront filters a strip of FS_S rows and
// 64 - 2 RF columns, where RF = npass + compensate.  Lane L holds column
// c0 + L - RF of every row.  The x passes take their neighbours from the
// adjacent lanes, the y passes from the rows held in registers.  The
// outermost lanes and rows take arbitrary values that move one cell inwards
// per pass, so after RF passes lanes [RF, 64 - RF) and rows [RF, FS_S + RF)
// are exact.  Same arithmetic as filter_body, term for term.
constexpr int FS_S = 8;

// The N + c passes of the filter on rows held in registers, one column per
// lane: x passes with the adjacent lanes' values (gap columns held at zero),
// then y passes along the rows.  Lanes and rows within RF of the edges end
// with arbitrary values.
template <typename R, int RF, int NR>
__device__ __forceinline__ void filter_rows(R (&a)[NR][3], bool gp, int npass)
{
#pragma clang fp contract(off)
    const R N = (R)npass;
#pragma unroll
    for (int pass = 0; pass < RF; ++pass) {
        const bool comp = pass == npass;
        const R w0 = comp ? -N / R(4) : R(0.25), w1 = comp ? (R(4) + R(2) * N) / R(4) : R(0.5);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R l = __shfl_up(a[q][c], 1), r = __shfl_down(a[q][c], 1);
                a[q][c] = gp ? R(0) : w0 * l + w1 * a[q][c] + w0 * r;
            }
        }
    }
#pragma unroll
    for (int pass = 0; pass < RF; ++pass) {
        const bool comp = pass == npass;
        const R w0 = comp ? -N / R(4) : R(0.25), w1 = comp ? (R(4) + R(2) * N) / R(4) : R(0.5);
        R b[NR][3];
#pragma unroll
        for (int q = 1; q < NR - 1; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) b[q][c] = w0 * a[q - 1][c] + w1 * a[q][c] + w0 * a[q + 1][c];
        }
#pragma unroll
        for (int q = 1; q < NR - 1; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a[q][c] = b[q][c];
        }
    }
}

template <typename R, int RF>
__global__ __launch_bounds__(64) void k_filter_s(SimDev<R> d, const R *i0, const R *i1,
                                                const R *i2, R *o0, R *o1, R *o2,
                                                int before_shift)
{
    constexpr int W = 64 - 2 * RF, NRW = FS_S + 2 * RF;
    const int ncg = (d.nxs + W - 1) / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int cg = blk % ncg, r0 = (blk / ncg) * FS_S;
    const int nr = min(FS_S, d.ny - r0);
    const int L = threadIdx.x;
    const int cx = cg * W + L - RF;
    int gx = cx % d.nxs;
    gx += gx < 0 ? d.nxs : 0;
    const bool put = L >= RF && L < 64 - RF && cx < d.nxs;
    // before_shift: the gap of the window the last step deposited in
    const int origin = wrapi(glob(d.st)->origin - (before_shift ? glob(d.st)->shift : 0), d.nxs);
    const bool gp = d.window && window_col(gx, origin, d.nxs) >= d.nx;
    auto at = [&](int j) {
        int gy = j % d.ny;
        gy += gy < 0 ? d.ny : 0;
        return (size_t)gx + (size_t)gy * d.nxs;
    };
    const gptr<const R> in[3] = {glob(i0), glob(i1), glob(i2)};
    R a[NRW][3];
#pragma unroll
    for (int q = 0; q < NRW; ++q) {
        const size_t g = at(r0 - RF + q);
#pragma unroll
        for (int c = 0; c < 3; ++c) a[q][c] = in[c][g];
    }
    filter_rows<R, RF>(a, gp, d.npass);
    R *const out[3] = {o0, o1, o2};
#pragma unroll
    for (int m = 0; m < FS_S; ++m) {
        if (put && m < nr) {
            const size_t g = at(r0 + m);
#pragma unroll
            for (int c = 0; c < 3; ++c) glob(out[c])[g] = a[RF + m][c];
        }
    }
}

// Rows a6 + a7 in streaming form, for one simulation: each wavefront filters
// the current and advances the fields on a strip of YS_S rows.  Lane L holds
// column c0 + L - P of every row, P = max(1, RF), so one row of a plane is a
// single contiguous load of the wavefront; x neighbours come from the
// adjacent lanes and y neighbours from the rows held in registers.  All loads
// of the strip go out before the first update.  With RF = npass + compensate
// > 0 the current is J filtered in registers (filter_rows, exact on lanes
// RF .. 63 - RF); with RF = 0 it is read as is.  The Yee halo is lane P - 1
// (B half at i - 1) and lanes beyond the strip (E at i + 1, i + 2): lanes
// P .. 62 - P end with complete results.  The arithmetic is that of
// filter_body and yee_body, term for term.
template <typename R, int RF, bool FOLD = false>
__device__ __forceinline__ void yee_s_body(const SimDev<R> &d, const int blk)
{
    // no contraction into fma: the tile and streaming forms (and the batched
    // launches) must round every term alike
#pragma clang fp contract(off)
    constexpr int P = RF > 1 ? RF : 1, W = yee_strip_w(RF);
    const int ncg = (d.nxs + W - 1) / W;
    const int cg = blk % ncg, r0 = (blk / ncg) * YS_S;
    const int nr = min(YS_S, d.ny - r0);
    const int L = threadIdx.x;
    const int cx = cg * W + L - P;
    int gx = cx % d.nxs;
    gx += gx < 0 ? d.nxs : 0;
    const bool put = L >= P && L < P + W && cx < d.nxs;
    const int par = glob(d.st)->parity, origin = glob(d.st)->origin;
    const bool gp = d.window && window_col(gx, origin, d.nxs) >= d.nx;
    const R hdt = R(0.5) * d.dt;
    auto at = [&](int j) {
        int gy = j % d.ny;
        gy += gy < 0 ? d.ny : 0;
        return (size_t)gx + (size_t)gy * d.nxs;
    };
    // rows r0 - 1 + q: E for q in [0, YS_S + 3), B in [0, YS_S + 2); the
    // current on rows r0 .. r0 + YS_S, filtered here from J (RF > 0: rows
    // r0 - RF .. r0 + YS_S + RF of J) or read as is
    constexpr int NJ = YS_S + 1 + 2 * RF;
    R eo[YS_S + 3][3], bo[YS_S + 2][3], ja[NJ][3];
#pragma unroll
    for (int q = 0; q < YS_S + 3; ++q) {
        const size_t g = at(r0 - 1 + q);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            eo[q][c] = glob<const R>(par ? d.F[1][c] : d.F[0][c])[g];
            if (q < YS_S + 2) bo[q][c] = glob<const R>(par ? d.F[1][3 + c] : d.F[0][3 + c])[g];
        }
    }
    if constexpr (FOLD) {
        // the current folded here from the tile images (fold_cell), and
        // written to J on the strip's own cells, as the fold launch would
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            int gy = (r0 - RF + q) % d.ny;
            gy += gy < 0 ? d.ny : 0;
            R v[3];
            fold_cell(d, gx, gy, v);
#pragma unroll
            for (int c = 0; c < 3; ++c) ja[q][c] = gp ? R(0) : v[c];
            const int m = q - RF;
            if (put && m >= 0 && m < nr) {
                const size_t g = (size_t)gx + (size_t)gy * d.nxs;
#pragma unroll
                for (int c = 0; c < 3; ++c) glob(d.J[c])[g] = ja[q][c];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const size_t g = at(r0 - RF + q);
#pragma unroll
            for (int c = 0; c < 3; ++c) ja[q][c] = glob<const R>(RF > 0 ? d.J[c] : d.Jf[c])[g];
        }
    }
    if constexpr (RF > 0) filter_rows<R, RF>(ja, gp, d.npass);
    R (&jj)[NJ][3] = ja;  // jj[RF + m]: row r0 + m
    // B half step, rows r0 - 1 .. r0 + YS_S
    R bh[YS_S + 2][3];
#pragma unroll
    for (int q = 0; q < YS_S + 2; ++q) {
        const R ey1 = __shfl_down(eo[q][1], 1), ez1 = __shfl_down(eo[q][2], 1);
        const R dEz_dy = (eo[q + 1][2] - eo[q][2]) * d.idy;
        const R dEz_dx = (ez1 - eo[q][2]) * d.idx;
        const R dEy_dx = (ey1 - eo[q][1]) * d.idx;
        const R dEx_dy = (eo[q + 1][0] - eo[q][0]) * d.idy;
        bh[q][0] = gp ? R(0) : bo[q][0] - hdt * dEz_dy;
        bh[q][1] = gp ? R(0) : bo[q][1] + hdt * dEz_dx;
        bh[q][2] = gp ? R(0) : bo[q][2] - hdt * (dEy_dx - dEx_dy);
    }
    // E full step, rows r0 .. r0 + YS_S
    R en[YS_S + 1][3];
#pragma unroll
    for (int q = 1; q < YS_S + 2; ++q) {
        const R by0 = __shfl_up(bh[q][1], 1), bz0 = __shfl_up(bh[q][2], 1);
        const R dBz_dy = (bh[q][2] - bh[q - 1][2]) * d.idy;
        const R dBz_dx = (bh[q][2] - bz0) * d.idx;
        const R dBy_dx = (bh[q][1] - by0) * d.idx;
        const R dBx_dy = (bh[q][0] - bh[q - 1][0]) * d.idy;
        en[q - 1][0] = gp ? R(0) : eo[q][0] + d.dt * (dBz_dy - jj[RF + q - 1][0]);
        en[q - 1][1] = gp ? R(0) : eo[q][1] + d.dt * (-dBz_dx - jj[RF + q - 1][1]);
        en[q - 1][2] = gp ? R(0) : eo[q][2] + d.dt * (dBy_dx - dBx_dy - jj[RF + q - 1][2]);
    }
    // B half step on the strip's rows, and write out
    const int npar = par ^ 1;
#pragma unroll
    for (int m = 0; m < YS_S; ++m) {
        const R ey1 = __shfl_down(en[m][1], 1), ez1 = __shfl_down(en[m][2], 1);
        const R dEz_dy = (en[m + 1][2] - en[m][2]) * d.idy;
        const R dEz_dx = (ez1 - en[m][2]) * d.idx;
        const R dEy_dx = (ey1 - en[m][1]) * d.idx;
        const R dEx_dy = (en[m + 1][0] - en[m][0]) * d.idy;
        const R nbx = gp ? R(0) : bh[m + 1][0] - hdt * dEz_dy;
        const R nby = gp ? R(0) : bh[m + 1][1] + hdt * dEz_dx;
        const R nbz = gp ? R(0) : bh[m + 1][2] - hdt * (dEy_dx - dEx_dy);
        if (put && m < nr) {
            const size_t g = at(r0 + m);
            glob(npar ? d.F[1][0] : d.F[0][0])[g] = en[m][0];
            glob(npar ? d.F[1][1] : d.F[0][1])[g] = en[m][1];
            glob(npar ? d.F[1][2] : d.F[0][2])[g] = en[m][2];
            glob(npar ? d.F[1][3] : d.F[0][3])[g] = nbx;
            glob(npar ? d.F[1][4] : d.F[0][4])[g] = nby;
            glob(npar ? d.F[1][5] : d.F[0][5])[g] = nbz;
        }
    }
}

// Work order of the push and the particle layouts: one block of NTO
// threads, launched at most every 8 pushes (k_order below).
constexpr int NTO = 1024;

// Block-wide sum of v over NTO threads (every thread gets the sum).
__device__ __forceinline__ long long block_sum_ll(long long v, long long *s_part)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) s_part[wv] = v;
    __syncthreads();
    long long t = 0;
    for (int k = 0; k < NTO / 64; ++k) t += s_part[k];
    return t;
}

// Exclusive prefix of v over NTO threads in thread order; *total gets the sum.
__device__ __forceinline__ long long block_prefix_ll(long long v, long long *s_part,
                                                     long long *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    long long inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    __syncthreads();
    if (lane == 63) s_part[wv] = inc;
    __syncthreads();
    long long before = 0, t = 0;
    for (int k = 0; k < NTO / 64; ++k) {
        before += k < wv ? s_part[k] : 0;
        t += s_part[k];
    }
    *total = t;
    return before + inc - v;
}

// Steps a layout must absorb: the layout is checked with the work order at
// the start of every 8-step graph, so up to 15 steps can pass between checks
// (8-step graphs and then up to 7 one-step graphs).
constexpr int GROW_STEPS = 16;

// Room tile t of species P needs in its segment to last GROW_STEPS more
// steps: its count, plus 64, plus twice what it gained since the last check,
// plus GROW_STEPS times what entered it from its neighbours in the last
// step (counted by the push, or by the hand-off that appended them), and
// with the moving window the columns loaded at the right edge meanwhile.
template <typename R>
__device__ __forceinline__ long long seg_need(const SimDev<R> &d, const SpDev<R> &P, int pp,
                                              int origin, int t)
{
    const int tx = t % d.ntx, ty = t / d.ntx;
    const long long cnt = glob(P.pb[pp].count)[t];
    const long long grown = cnt - glob(P.snap)[t];
    long long need = cnt + 64 + (grown > 0 ? 2 * grown : 0);
    // what entered it in the last step that moved particles between tiles,
    // for every step until the next check
    need += (long long)GROW_STEPS * glob(P.inflow)[t];
    if (d.window && P.density > 0.0) {
        // storage columns entering over the next GROW_STEPS steps (at most
        // one per step, since dt < dx)
        const int first = (origin + d.nx) % d.nxs;
        const int x0 = tx * TX, w = min(TX, d.nxs - x0), h = min(TY, d.ny - ty * TY);
        int cols = 0;
        for (int c = 0; c < GROW_STEPS; ++c) {
            const int gx = (first + c) % d.nxs;
            cols += gx >= x0 && gx < x0 + w;
        }
        need += (long long)cols * h * P.ppc_x * P.ppc_y;
    }
    return need;
}

// Relayout of species s's buffer ppar ^ 1 if some tile's need exceeds its
// segment in buffer ppar: each tile gets its need rounded up to 64 slots,
// plus a share of the rest of the pool in proportion to count + average
// count (so that empty tiles can take in a front), at most maxseg; the
// segments are laid out in tile order (a block-wide scan per row of NTO
// tiles).  The next push writes its output at
// this layout.  A pool too small for the needs raises the capacity error
// and keeps the layout.  Every tile's count is kept as its snapshot for the
// next check.  *s_flag must be zero, with a barrier, on entry.
template <typename R>
__device__ void relayout_body(const SimDev<R> &d, int s, long long *s_part, int *s_flag)
{
    const SpDev<R> &P = d.sp[s];
    const gptr<const DevState> st = glob<const DevState>(d.st);
    const int pp = st->ppar, origin = st->origin;
    const int n = d.ntiles, rows = (n + NTO - 1) / NTO;
    const gptr<int> needv = glob(P.need);
    const gptr<const int> cnt_a = glob<const int>(P.pb[pp].count);
    // tiles t = r * NTO + thread, so that every load of a row is coalesced;
    // rows in groups of RG whose loads all go out before the group's stores
    constexpr int RG = 4;
    long long cnt = 0, nd = 0;
    bool tight = false;
    for (int r0 = 0; r0 < rows; r0 += RG) {
        long long need[RG];
        int cn[RG], sl[RG];
#pragma unroll
        for (int k = 0; k < RG; ++k) {
            const int t = (r0 + k) * NTO + (int)threadIdx.x;
            need[k] = 0;
            cn[k] = 0;
            sl[k] = 0;
            if (r0 + k < rows && t < n) {
                need[k] = seg_need(d, P, pp, origin, t);
                cn[k] = cnt_a[t];
                sl[k] = seg_slots(P, pp, t);
            }
        }
#pragma unroll
        for (int k = 0; k < RG; ++k) {
            const int t = (r0 + k) * NTO + (int)threadIdx.x;
            if (r0 + k < rows && t < n) {
                const long long base = min((long long)P.maxseg, (need[k] + 63) / 64 * 64);
                needv[t] = (int)base;
                glob(P.snap)[t] = cn[k];  // the count, for the growth seen at the next check
                cnt += cn[k];
                nd += base;
                tight |= need[k] > sl[k];
            }
        }
    }
    if (tight) *s_flag = 1;  // plain store: any thread may set it
    const long long total_cnt = block_sum_ll(cnt, s_part);
    const long long total_need = block_sum_ll(nd, s_part);
    if (!*s_flag) return;  // block-uniform (read after the barriers above)
    const long long spare = (long long)P.pool - total_need;
    if (spare < 0) {
        if (threadIdx.x == 0)
            __hip_atomic_fetch_or(&glob(d.st)->err, ERR_POOL, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const double avg = (double)total_cnt / n;
    const double wsum = (double)total_cnt + avg * n;
    long long run = 0;  // slots of the rows before (block-uniform)
    for (int r = 0; r < rows; ++r) {
        const int t = r * NTO + (int)threadIdx.x;
        long long cap = 0;
        if (t < n) {
            const double wt = (double)cnt_a[t] + avg;
            const long long share = wsum > 0 ? (long long)((double)spare * wt / wsum) / 64 * 64 : 0;
            cap = min((long long)P.maxseg, (long long)needv[t] + share);
        }
        long long row;
        const long long ex = block_prefix_ll(cap, s_part, &row);
        if (t < n) {
            glob(P.start[pp ^ 1])[t] = run + ex;
            glob(P.seg[pp ^ 1])[t] = (int)cap;
        }
        run += row;
    }
}

// The push's block b takes work item order[b].  The items are sorted,
// heaviest first, into 64 load buckets, two per octave, with the bucket
// edges a quarter octave off the powers of two (a tile of 2^k particles, the
// usual initial load, sits mid-bucket, so sampling noise does not split such
// tiles over two buckets).  The sort is stable: within a bucket the items
// keep their tile order.  Blocks go to the 8 XCDs in turn (b % 8), each XCD
// with an L2 of its own, and the sorted list is dealt to them in chunks of
// ORDER_CHUNK consecutive items, so each XCD starts on the heavy items and
// works along runs of neighbouring tiles, which share field and current
// halos.
constexpr int ORDER_CHUNK = 8;

// Block of sorted position p (a bijection of [0, n)): chunks of ORDER_CHUNK
// positions dealt to the 8 XCDs in turn; the last, partial round ranked by
// (offset in chunk, chunk).
__device__ __forceinline__ int order_block(int p, int n)
{
    constexpr int G = ORDER_CHUNK, RND = 8 * ORDER_CHUNK;
    const int full = (n / RND) * RND;
    if (p < full) {
        // rounds of 8 chunks, the XCDs taking them forwards in even rounds
        // and backwards in odd ones (a heavy chunk, then a light one)
        const int rd = p / RND, c = (p / G) % 8, x = rd & 1 ? 7 - c : c;
        return 8 * (rd * G + p % G) + x;
    }
    const int T = n - full, q = p - full, x = q / G, o = q % G;
    const int nch = (T + G - 1) / G;
    int rank = 0;
    for (int c = 0; c < nch; ++c) {
        const int sz = min(G, T - c * G);
        rank += min(sz, o) + (c < x && sz > o ? 1 : 0);
    }
    return full + rank;
}

template <typename R>
__device__ __forceinline__ int item_load(const SimDev<R> &d, int pp, int i)
{
    const int t = i / d.nsb;
    if (d.nsb > 1) return glob(d.sp[i % d.nsb].pb[pp].count)[t];
    int n = 0;
    for (int s = 0; s < d.nsp; ++s) n += glob(d.sp[s].pb[pp].count)[t];
    return n;
}

__device__ __forceinline__ int load_bucket(int w)
{
    // 63 - floor(2 log2(w + 1) + 1/2): 0 for the heaviest, monotone
    const int k = (int)floorf(2.0f * __log2f((float)w + 1.0f) + 0.5f);
    return 63 - min(63, max(0, k));
}

// The particle layout of species s of one simulation (relayout_body).  One
// block of NTO threads; ends with a barrier.
template <typename R>
__device__ void layout_body(const SimDev<R> &d, int s)
{
    __shared__ long long s_part[NTO / 64];
    __shared__ int s_flag;
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    relayout_body(d, s, s_part, &s_flag);
    __syncthreads();
}

// The particle layouts of every species, one after another.
template <typename R>
__device__ void layouts_body(const SimDev<R> &d)
{
    for (int s = 0; s < d.nsp; ++s) layout_body(d, s);
}

// The push's work order from the tiles' counts.  One block of NTO threads.
template <typename R>
__device__ __forceinline__ void order_body(const SimDev<R> &d)
{
    __shared__ int s_wc[NTO / 64][64];
    __shared__ int s_base[64];
    // bucket of every item while they fit (read once, used by both passes)
    constexpr int KB_MAX = 16384;
    __shared__ unsigned char s_kb[KB_MAX];
    const int pp = glob(d.st)->ppar, n = d.ntiles * d.nsb;
    const int rows = (n + NTO - 1) / NTO;
    if (threadIdx.x < 64) s_base[threadIdx.x] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += 4 * NTO) {
        int kk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * NTO + (int)threadIdx.x;
            kk[k] = i < n ? load_bucket(item_load(d, pp, i)) : -1;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * NTO + (int)threadIdx.x;
            if (kk[k] >= 0 && n <= KB_MAX) s_kb[i] = (unsigned char)kk[k];
            // one LDS atomic per bucket present in the wavefront (most items
            // share a bucket: one atomic per lane would serialise on it)
            unsigned long long todo = __ballot(kk[k] >= 0);
            while (todo) {
                const int lead = __ffsll((long long)todo) - 1;
                const int kc = __shfl(kk[k], lead, 64);
                const unsigned long long m = __ballot(kk[k] == kc);
                if ((int)(threadIdx.x & 63) == lead) atomicAdd(&s_base[kc], (int)__popcll(m));
                todo &= ~m;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // exclusive prefix over the buckets, in one wavefront
        const int c = s_base[threadIdx.x];
        int v = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o, 64);
            if ((int)threadIdx.x >= o) v += u;
        }
        s_base[threadIdx.x] = v - c;
    }
    // stable counting sort, one row of NTO items at a time: the rank within
    // the wavefront by ballots over the buckets present in it, then the
    // counts of the wavefronts before
    const gptr<int> order = glob(d.order);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < rows; ++r) {
        const int i = r * NTO + (int)threadIdx.x;
        s_wc[wv][lane] = 0;
        __syncthreads();
        const int k = i >= n ? -1 : n <= KB_MAX ? (int)s_kb[i] : load_bucket(item_load(d, pp, i));
        int rank = 0;
        unsigned long long todo = __ballot(k >= 0);
        while (todo) {
            const int lead = __ffsll((long long)todo) - 1;
            const int kc = __shfl(k, lead, 64);
            const unsigned long long m = __ballot(k == kc);
            if (k == kc) rank = (int)__popcll(m & below);
            if (lane == lead) s_wc[wv][kc] = (int)__popcll(m);
            todo &= ~m;
        }
        __syncthreads();
        if (k >= 0) {
            int pos = s_base[k] + rank;
            for (int w2 = 0; w2 < wv; ++w2) pos += s_wc[w2][k];
            order[order_block(pos, n)] = i;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            int add = 0;
            for (int w2 = 0; w2 < NTO / 64; ++w2) add += s_wc[w2][threadIdx.x];
            s_base[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

// Blocks 0 .. nsp-1 lay out the particle segments of species blockIdx.x;
// block nsp writes the work order.  The parts run side by side: the order
// reads only the tiles' counts, which a relayout leaves as they are.
template <typename R>
__global__ __launch_bounds__(NTO) void k_order(SimDev<R> d)
{
    if ((int)blockIdx.x < d.nsp)
        layout_body(d, (int)blockIdx.x);
    else
        order_body(d);
}

// The particle layouts of every simulation of a batch, one block each.  The
// batched push takes its work from a (simulation, tile) list, so the
// simulations' own work orders are left as they are.
template <typename R>
__global__ __launch_bounds__(NTO) void k_layout_b(const SimDev<R> *__restrict__ ds)
{
    layouts_body(ds[blockIdx.x]);
}

template <typename R, int RF>
__global__ __launch_bounds__(64) void k_yee_s(SimDev<R> d)
{
    yee_s_body<R, RF>(d, xcd_remap(blockIdx.x, gridDim.x));
}

// rows a5-a7 in one launch: the fold of the tile images as well (one block
// per tile and float images, reduction deposit)
template <typename R, int RF>
__global__ __launch_bounds__(64) void k_fold_yee_s(SimDev<R> d)
{
    yee_s_body<R, RF, true>(d, xcd_remap(blockIdx.x, gridDim.x));
}

// the same over a batch whose simulations share the filter halo RF
template <typename R, int RF>
__global__ __launch_bounds__(64) void k_yee_sb(const SimDev<R> *__restrict__ ds,
                                               const BatchDev *__restrict__ b)
{
    const int n = __builtin_amdgcn_readfirstlane(b->nyee);
    if ((int)blockIdx.x >= n) return;
    const int2 w = b->yee_work[xcd_remap(blockIdx.x, n)];
    yee_s_body<R, RF>(ds[__builtin_amdgcn_readfirstlane(w.x)], __builtin_amdgcn_readfirstlane(w.y));
}

// True in thread 0 of the block that finishes a launch last: every block
// counts itself in *counter once all its threads are done; the last one
// resets the counter for the next launch and does the launch's closing work.
// No other block reads what that work changes (all have finished), and the
// next launch sees it at the kernel boundary, so the count needs no ordering
// beyond atomicity: relaxed device-scope atomics, which on this GPU do not
// write back or invalidate the XCD's L2 as acquire/release ones would.
__device__ __forceinline__ bool last_block(int *counter)
{
    __syncthreads();
    if (threadIdx.x != 0) return false;
    const int prev = __hip_atomic_fetch_add(glob(counter), 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    if (prev != (int)gridDim.x - 1) return false;
    __hip_atomic_store(glob(counter), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// ---------------------------------------------------------------------------
// end of step: flip the field buffers, count the step and decide the window
// shift (the window advances one cell once iter*dt >= (nshift+1)*dx, in double)
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void step_end_body(const SimDev<R> &d)
{
    DevState *st = d.st;
    st->parity ^= 1;
    st->iter += 1;
    st->shift = 0;
    if (d.window && (double)st->iter * d.dt_d >= (double)(st->nshift + 1) * d.dx_d) {
        st->shift = 1;
        st->nshift += 1;
        st->origin = wrapi(st->origin + 1, d.nxs);
    }
}

// Row a8, part 1 (blocks [0, nty*nsp)): particles of the column that left the
// window are removed by a stable in-tile compaction; part 2 (block nty*nsp):
// the six field planes of that column are cleared.  No-op unless shifted.
// With unpend, the field block also clears the pending flag of a hand-off
// that k_settle has just completed.
template <typename R>
__device__ __forceinline__ void window_clear_body(const SimDev<R> &d, const int blk, bool unpend)
{
    __shared__ int s_w[NT / 64];
    DevState *st = d.st;
    if (!st->shift) return;
    const int col = wrapi(st->origin - 1, d.nxs);
    const int par = st->parity;
    if (blk == d.nty * d.nsp) {
        if (unpend && threadIdx.x == 0) st->pend = 0;
        for (int j = threadIdx.x; j < d.ny; j += NT) {
            const size_t g = (size_t)col + (size_t)j * d.nxs;
#pragma unroll
            for (int c = 0; c < 6; ++c) (par ? d.F[1][c] : d.F[0][c])[g] = R(0);
        }
        return;
    }
    const int ty = blk % d.nty, s = blk / d.nty;
    const int t = col / TX + ty * d.ntx;
    const SpDev<R> &S = d.sp[s];
    const PartBuf<R> &P = S.pb[st->ppar];
    const size_t base = seg_start(S, st->ppar, t);
    const int n = P.count[t];
    int kept = 0;
    for (int p0 = 0; p0 < n; p0 += NT) {
        const int p = p0 + threadIdx.x;
        int c = 0;
        R x = 0, y = 0, ux = 0, uy = 0, uz = 0;
        bool keep = false;
        if (p < n) {
            c = P.cell[base + p];
            keep = cell_x(c) != col;
            x = P.x[base + p];
            y = P.y[base + p];
            ux = P.ux[base + p];
            uy = P.uy[base + p];
            uz = P.uz[base + p];
        }
        int tot;
        const int r = block_rank(keep, s_w, &tot);
        if (keep) {
            const size_t q = base + kept + r;
            P.cell[q] = c;
            P.x[q] = x;
            P.y[q] = y;
            P.ux[q] = ux;
            P.uy[q] = uy;
            P.uz[q] = uz;
        }
        kept += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) P.count[t] = kept;
}

template <typename R>
__global__ __launch_bounds__(NT) void k_window_clear(SimDev<R> d)
{
    window_clear_body(d, blockIdx.x, false);
}

// Row a8, part 3: load the column that entered at the right edge.
template <typename R>
__device__ __forceinline__ void window_inject_body(const SimDev<R> &d, const int blk)
{
    __shared__ int s_w[NT / 64];
    const DevState *st = d.st;
    if (!st->shift) return;
    const int col = wrapi(st->origin + d.nx - 1, d.nxs);
    const long long ilab = (long long)d.nx - 1 + st->nshift;
    const int ty = blk % d.nty, s = blk / d.nty;
    const int t = col / TX + ty * d.ntx;
    const int y0 = ty * TY, h = min(TY, d.ny - y0);
    const SpDev<R> &S = d.sp[s];
    if (!(S.density > 0.0)) return;
    const PartBuf<R> &P = S.pb[st->ppar];
    const int cap = seg_slots(S, st->ppar, t);
    const size_t base = seg_start(S, st->ppar, t);
    const int n0 = P.count[t];
    const int ppc = S.ppc_x * S.ppc_y;
    const int total = h * ppc;
    int added = 0;
    for (int q0 = 0; q0 < total; q0 += NT) {
        const int q = q0 + threadIdx.x;
        bool ok = false;
        int j = 0, m = 0, l = 0;
        if (q < total) {
            const int sub = q / h;
            j = y0 + q % h;
            m = sub % S.ppc_x;
            l = sub / S.ppc_x;
            const double xo = ((double)m + 0.5) / (double)S.ppc_x;
            const double xlab = ((double)ilab + xo) * d.dx_d;
            ok = xlab >= S.x_lo && xlab < S.x_hi;
        }
        int tot;
        const int r = block_rank(ok, s_w, &tot);
        if (ok) {
            const int pos = n0 + added + r;
            if (pos < cap) {
                R u[3];
                maxwellian(S, d.key0, d.key1, (uint32_t)ilab, (uint32_t)j,
                           (uint32_t)(l * S.ppc_x + m), (uint32_t)s, u);
                const size_t o = base + pos;
                P.cell[o] = pack_cell(col, j);
                P.x[o] = (R)(((double)m + 0.5) / (double)S.ppc_x);
                P.y[o] = (R)(((double)l + 0.5) / (double)S.ppc_y);
                P.ux[o] = u[0];
                P.uy[o] = u[1];
                P.uz[o] = u[2];
            } else {
                atomicOr(&d.st->err, ERR_INJECT);
            }
        }
        added += tot;
    }
    if (threadIdx.x == 0) P.count[t] = min(n0 + added, cap);
}

template <typename R>
__global__ __launch_bounds__(NT) void k_window_inject(SimDev<R> d)
{
    window_inject_body(d, blockIdx.x);
}

// Both parts of the shift in one launch, and the pending flag of the
// preceding hand-off cleared: blocks [0, nty*nsp] clear, the rest inject.
// The leaving and the entering column lie at least nx cells apart both ways
// round the ring, so with nx >= 16 they are in different tiles.
template <typename R>
__global__ __launch_bounds__(NT) void k_window(SimDev<R> d)
{
    const int a = d.nty * d.nsp;
    if ((int)blockIdx.x <= a)
        window_clear_body(d, blockIdx.x, true);
    else
        window_inject_body(d, (int)blockIdx.x - a - 1);
}

// Initial load of species s, one block per tile.  Particles are stored
// sub-position major, cell minor, so that consecutive particles (one
// wavefront) sit in different cells and their LDS atomics rarely collide.
template <typename R>
__global__ __launch_bounds__(NT) void k_load(SimDev<R> d, int s)
{
    __shared__ int s_w[NT / 64];
    const int t = blockIdx.x;
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    const SpDev<R> &S = d.sp[s];
    const PartBuf<R> &P = S.pb[d.st->ppar];
    const int origin = d.st->origin, nshift = d.st->nshift;
    const int cap = seg_slots(S, d.st->ppar, t);
    const size_t base = seg_start(S, d.st->ppar, t);
    const int ncell = w * h, ppc = S.ppc_x * S.ppc_y;
    const int total = ncell * ppc;
    int added = 0;
    for (int q0 = 0; q0 < total; q0 += NT) {
        const int q = q0 + threadIdx.x;
        bool ok = false;
        int gx = 0, gy = 0, m = 0, l = 0;
        long long ilab = 0;
        if (q < total && S.density > 0.0) {
            const int sub = q / ncell, c = q % ncell;
            gx = x0 + c % w;
            gy = y0 + c / w;
            m = sub % S.ppc_x;
            l = sub / S.ppc_x;
            const int wc = d.window ? window_col(gx, origin, d.nxs) : gx;
            ilab = (long long)wc + nshift;
            const double xo = ((double)m + 0.5) / (double)S.ppc_x;
            const double xlab = ((double)ilab + xo) * d.dx_d;
            ok = wc < d.nx && xlab >= S.x_lo && xlab < S.x_hi;
        }
        int tot;
        const int r = block_rank(ok, s_w, &tot);
        if (ok) {
            const int pos = added + r;
            if (pos < cap) {
                R u[3];
                maxwellian(S, d.key0, d.key1, (uint32_t)ilab, (uint32_t)gy,
                           (uint32_t)(l * S.ppc_x + m), (uint32_t)s, u);
                const size_t o = base + pos;
                P.cell[o] = pack_cell(gx, gy);
                P.x[o] = (R)(((double)m + 0.5) / (double)S.ppc_x);
                P.y[o] = (R)(((double)l + 0.5) / (double)S.ppc_y);
                P.ux[o] = u[0];
                P.uy[o] = u[1];
                P.uz[o] = u[2];
            } else {
                atomicOr(&d.st->err, ERR_LOAD);
            }
        }
        added += tot;
    }
    if (threadIdx.x == 0) P.count[t] = min(added, cap);
}

// ---------------------------------------------------------------------------
// row a9: diagnostics (FP64 reductions)
// ---------------------------------------------------------------------------
// charge density on the nodes: per-tile LDS deposit of bilinear weights,
// flushed to plane 0 of the tile blocks (folded afterwards)
template <typename R>
__global__ __launch_bounds__(NT) void k_rho(SimDev<R> d)
{
    __shared__ unsigned long long sr[BP];
    const int t = blockIdx.x;
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    for (int k = threadIdx.x; k < BP; k += NT) sr[k] = 0ull;
    __syncthreads();
    for (int s = 0; s < d.nsp; ++s) {
        const SpDev<R> &S = d.sp[s];
        const PartBuf<R> &P = S.pb[d.st->ppar];
        const int n = P.count[t];
        const size_t base = seg_start(S, d.st->ppar, t);
        const R qp = S.qp * d.jq;  // carries the fixed-point scale
        for (int p = threadIdx.x; p < n; p += NT) {
            const int c = P.cell[base + p];
            const R x = P.x[base + p], y = P.y[base + p];
            const int k = (cell_x(c) - x0 + 1) + (cell_y(c) - y0 + 1) * PX;
            lds_acc(sr + k, qp * (R(1) - x) * (R(1) - y));
            lds_acc(sr + k + 1, qp * x * (R(1) - y));
            lds_acc(sr + k + PX, qp * (R(1) - x) * y);
            lds_acc(sr + k + PX + 1, qp * x * y);
        }
    }
    __syncthreads();
    R *out = d.blk + (size_t)t * 3 * BP;
    for (int k = threadIdx.x; k < BP; k += NT) out[k] = (R)fx_value(sr[k], d.jq_inv);
}

template <typename R>
__device__ __forceinline__ double div_at(const R *fx, const R *fy, const SimDev<R> &d, int gx,
                                         int gy, int origin)
{
    // backward differences at node (gx, gy) of an (x-staggered, y-staggered)
    // pair; values beyond the window are zero
    const int xm = wrapi(gx - 1, d.nxs), ym = wrapi(gy - 1, d.ny);
    const size_t g = (size_t)gx + (size_t)gy * d.nxs;
    double vxm = (double)fx[(size_t)xm + (size_t)gy * d.nxs];
    if (d.window && window_col(xm, origin, d.nxs) >= d.nx) vxm = 0.0;
    return ((double)fx[g] - vxm) / d.dx_d +
           ((double)fy[g] - (double)fy[(size_t)gx + (size_t)ym * d.nxs]) / d.dy_d;
}

// g0 = div E^0 - F rho^0 (rho_f must hold F rho^0)
template <typename R>
__global__ __launch_bounds__(NT) void k_g0(SimDev<R> d)
{
    const int par = d.st->parity, origin = d.st->origin;
    const R *ex = par ? d.F[1][0] : d.F[0][0];
    const R *ey = par ? d.F[1][1] : d.F[0][1];
    const long long ncell = (long long)d.nxs * d.ny;
    for (long long g = blockIdx.x * (long long)NT + threadIdx.x; g < ncell;
         g += (long long)gridDim.x * NT) {
        const int gx = (int)(g % d.nxs), gy = (int)(g / d.nxs);
        const bool gap = d.window && window_col(gx, origin, d.nxs) >= d.nx;
        d.g0[g] = gap ? 0.0 : div_at(ex, ey, d, gx, gy, origin) - (double)d.rho_f[g];
    }
}

__device__ double block_sum(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// field energy and the Gauss / continuity residuals, per block partials:
// red[b*5 + {0: E^2, 1: B^2, 2: gauss max, 3: continuity max, 4: |rho| max}]
template <typename R>
__global__ __launch_bounds__(NT) void k_diag_grid(SimDev<R> d, int has_prev)
{
    __shared__ double sred[NT];
    const int par = d.st->parity, origin = d.st->origin;
    // With the moving window the residuals skip the columns next to the left
    // edge (particles leave there and the fields beyond are held at zero) and
    // the columns loaded since t = 0 (their neutralising background is not in
    // the t = 0 baseline), each with a margin for the filter and the weights.
    const int res_lo = 3, res_hi = d.nx - d.st->nshift - 3;
    const R *F[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) F[c] = par ? d.F[1][c] : d.F[0][c];
    const long long ncell = (long long)d.nxs * d.ny;
    double e2 = 0, b2 = 0, gm = 0, cm = 0, rm = 0;
    const double idt = 1.0 / d.dt_d;
    for (long long g = blockIdx.x * (long long)NT + threadIdx.x; g < ncell;
         g += (long long)gridDim.x * NT) {
        const int gx = (int)(g % d.nxs), gy = (int)(g / d.nxs);
        const int wc = d.window ? window_col(gx, origin, d.nxs) : 0;
        if (d.window && wc >= d.nx) continue;
        const double ex = F[0][g], ey = F[1][g], ez = F[2][g];
        const double bx = F[3][g], by = F[4][g], bz = F[5][g];
        e2 += ex * ex + ey * ey + ez * ez;
        b2 += bx * bx + by * by + bz * bz;
        rm = fmax(rm, fabs((double)d.rho[g]));
        if (d.window && (wc < res_lo || wc >= res_hi)) continue;
        const double gres = div_at(F[0], F[1], d, gx, gy, origin) - (double)d.rho_f[g] - d.g0[g];
        gm = fmax(gm, fabs(gres));
        if (has_prev) {
            const double cres = ((double)d.rho[g] - (double)d.rho_prev[g]) * idt +
                                div_at(d.J[0], d.J[1], d, gx, gy, origin);
            cm = fmax(cm, fabs(cres));
        }
    }
    e2 = block_sum(e2, sred);
    b2 = block_sum(b2, sred);
    gm = block_max(gm, sred);
    cm = block_max(cm, sred);
    rm = block_max(rm, sred);
    if (threadIdx.x == 0) {
        double *r = d.red + (size_t)blockIdx.x * 5;
        r[0] = e2;
        r[1] = b2;
        r[2] = gm;
        r[3] = cm;
        r[4] = rm;
    }
}

// kinetic energy per tile and species with u- = u + (q/m)(dt/2) E^n(x^n):
// red[NB_DIAG*5 + t*MAX_SP + s]
template <typename R>
__global__ __launch_bounds__(NT) void k_diag_ke(SimDev<R> d)
{
    __shared__ R sf[6 * BP];
    __shared__ double sred[NT];
    const int t = blockIdx.x;
    const int tx = t % d.ntx, ty = t / d.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = min(TX, d.nxs - x0), h = min(TY, d.ny - y0);
    load_tile_fields<NT>(d, d.st->parity, x0, y0, w, h, sf, (unsigned long long *)nullptr);
    __syncthreads();
    for (int s = 0; s < d.nsp; ++s) {
        const SpDev<R> &S = d.sp[s];
        const PartBuf<R> &P = S.pb[d.st->ppar];
        const int n = P.count[t];
        const size_t base = seg_start(S, d.st->ppar, t);
        const double mp = (double)S.qp / (double)S.qm;
        double ke = 0;
        for (int p = threadIdx.x; p < n; p += NT) {
            const int c = P.cell[base + p];
            const R x = P.x[base + p], y = P.y[base + p];
            const int lx = cell_x(c) - x0, ly = cell_y(c) - y0;
            const bool lox = x < R(0.5), loy = y < R(0.5);
            const int ixh = lx - (lox ? 1 : 0), iyh = ly - (loy ? 1 : 0);
            const R wxh = x + (lox ? R(0.5) : R(-0.5)), wyh = y + (loy ? R(0.5) : R(-0.5));
            const double ex = lerp2(sf, ixh, ly, wxh, y);
            const double ey = lerp2(sf + BP, lx, iyh, x, wyh);
            const double ez = lerp2(sf + 2 * BP, lx, ly, x, y);
            const double tau = (double)S.tau;
            const double a = (double)P.ux[base + p] + tau * ex;
            const double b = (double)P.uy[base + p] + tau * ey;
            const double cc = (double)P.uz[base + p] + tau * ez;
            const double u2 = a * a + b * b + cc * cc;
            ke += mp * u2 / (sqrt(1.0 + u2) + 1.0);
        }
        ke = block_sum(ke, sred);
        if (threadIdx.x == 0) d.red[(size_t)NB_DIAG * 5 + (size_t)t * MAX_SP + s] = ke;
    }
}

// final fixed-order reduction of the partials into d.res:
// [0] E energy, [1] B energy, [2..5] KE per species, [6] gauss max,
// [7] continuity max, [8] |rho| max
template <typename R>
__global__ __launch_bounds__(NT) void k_diag_final(SimDev<R> d)
{
    __shared__ double sred[NT];
    const double area = d.dx_d * d.dy_d;
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < NB_DIAG; b += NT) {
        const double *r = d.red + (size_t)b * 5;
        v[0] += r[0];
        v[1] += r[1];
        v[2] = fmax(v[2], r[2]);
        v[3] = fmax(v[3], r[3]);
        v[4] = fmax(v[4], r[4]);
    }
    const double e2 = block_sum(v[0], sred), b2 = block_sum(v[1], sred);
    const double gm = block_max(v[2], sred), cm = block_max(v[3], sred);
    const double rm = block_max(v[4], sred);
    for (int s = 0; s < d.nsp; ++s) {
        double k = 0;
        for (int t = threadIdx.x; t < d.ntiles; t += NT)
            k += d.red[(size_t)NB_DIAG * 5 + (size_t)t * MAX_SP + s];
        k = block_sum(k, sred);
        if (threadIdx.x == 0) d.res[2 + s] = k * area;
    }
    if (threadIdx.x == 0) {
        d.res[0] = 0.5 * e2 * area;
        d.res[1] = 0.5 * b2 * area;
        d.res[6] = gm;
        d.res[7] = cm;
        d.res[8] = rm;
    }
}

template <typename R>
__global__ void k_copy(const R *src, R *dst, long long n)
{
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// kernels of one step: one simulation (descriptor in the kernel arguments,
// one block per tile), or a batch of simulations (descriptor table and a
// (simulation, tile) work list in device memory; blocks past the work count
// exit, so one captured graph serves every batch that fits its grid)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool batch_item(const BatchDev *__restrict__ b, int2 *item)
{
    const int nw = __builtin_amdgcn_readfirstlane(b->nwork);
    if ((int)blockIdx.x >= nw) return false;
    const int2 w = b->work[xcd_remap(blockIdx.x, nw)];
    // block-uniform: keep the descriptor address in scalar registers
    item->x = __builtin_amdgcn_readfirstlane(w.x);
    item->y = __builtin_amdgcn_readfirstlane(w.y);
    return true;
}



// Waves per SIMD the single-simulation push is compiled for: FP32 fits four
// 512-thread blocks per CU in 64 VGPRs; FP64 needs more registers.  Blocks of
// 512 threads halve the time one tile occupies its CU, which shortens the
// drain at the end of the launch, when too few tiles are left to fill the GPU.
template <typename R> struct PushWaves { static constexpr int n = 8; };
template <> struct PushWaves<double> { static constexpr int n = 4; };

// Tiles that hold many particles (the Weibel run's 131,072) take blocks of
// NTP_BIG threads: a tile's work then spreads over twice the wavefronts,
// which shortens the launch most when the particles pile up in a few tiles.
//
// Block b takes work item d.order[b] (a tile, or a tile's species block).
// Blocks are dispatched in about the order of their index, and k_order
// (at most every 8 steps) sorts the items heaviest first in load buckets and
// deals them to the XCDs in runs of neighbours, so heavy tiles start first
// and the launch ends on light ones: the GPU form of the paper's
// over-decomposition with dynamic distribution of regions to workers
// (Sec. 3.2, 4.3), where a region that holds many particles must not start
// last.
template <typename R, int BT>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(PushWaves<R>::n))) void
k_push_deposit(SimDev<R> d)
{
    __shared__ PushShared<R, ArrivalCap<BT>::n> sh;
    const int nsb = d.nsb;
    const int i = __builtin_amdgcn_readfirstlane(glob(d.order)[blockIdx.x]);
    push_counters_zero(sh);
    __syncthreads();
    push_tile<BT, false>(d, i / nsb, i % nsb, nsb, sh);
    if (last_block(&d.st->blocks_done)) push_end_body(d);
}

template <typename R>
__global__ __launch_bounds__(NTB) __attribute__((amdgpu_waves_per_eu(PushWaves<R>::n))) void
k_push_deposit_b(const SimDev<R> *__restrict__ ds,
                                             const BatchDev *__restrict__ b)
{
    int2 it;
    if (batch_item(b, &it)) push_body<NTB, false>(ds[it.x], it.y);
    if (last_block(&const_cast<BatchDev *>(b)->blocks_done))
        for (int i = 0; i < b->nsim; ++i) push_end_body(ds[i]);
}

// The commutative deposit: one launch per checkerboard colour (tiles with
// tx % 2 == colour & 1 and ty % 2 == colour >> 1) adds its tiles' current
// straight into J; the launch of the last colour flips the particle buffers.
template <typename R>
__global__ __launch_bounds__(NTP) __attribute__((amdgpu_waves_per_eu(PushWaves<R>::n))) void
k_push_colour(SimDev<R> d, int colour)
{
    const int hx = d.ntx >> 1;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = 2 * (i % hx) + (colour & 1), ty = 2 * (i / hx) + (colour >> 1);
    push_body<NTP, true>(d, tx + ty * d.ntx);
    if (last_block(&d.st->blocks_done) && colour == 3) push_end_body(d);
}

// J = 0 on the three planes before the first colour
template <typename R>
__global__ __launch_bounds__(NT) void k_zero_j(SimDev<R> d)
{
    const long long n = (long long)d.nxs * d.ny;
    for (long long g = blockIdx.x * (long long)NT + threadIdx.x; g < n;
         g += (long long)gridDim.x * NT) {
        glob(d.J[0])[g] = R(0);
        glob(d.J[1])[g] = R(0);
        glob(d.J[2])[g] = R(0);
    }
}

template <typename R>
__global__ __launch_bounds__(NT) void k_fold(SimDev<R> d, int nplanes, R *o0, R *o1, R *o2)
{
    fold_body(d, xcd_remap(blockIdx.x, gridDim.x), nplanes, o0, o1, o2);
}

template <typename R>
__global__ __launch_bounds__(NT) void k_fold_b(const SimDev<R> *__restrict__ ds,
                                             const BatchDev *__restrict__ b)
{
    int2 it;
    if (!batch_item(b, &it)) return;
    const SimDev<R> &d = ds[it.x];
    fold_body(d, it.y, 3, d.J[0], d.J[1], d.J[2]);
}

template <typename R>
__global__ __launch_bounds__(NT) void k_filter(SimDev<R> d, int nplanes, const R *i0,
                                               const R *i1, const R *i2, R *o0, R *o1, R *o2)
{
    filter_body(d, xcd_remap(blockIdx.x, gridDim.x), nplanes, i0, i1, i2, o0, o1, o2);
}

template <typename R>
__global__ __launch_bounds__(NT) void k_filter_b(const SimDev<R> *__restrict__ ds,
                                             const BatchDev *__restrict__ b)
{
    int2 it;
    if (!batch_item(b, &it)) return;
    const SimDev<R> &d = ds[it.x];
    if (d.npass == 0) return;
    filter_body(d, it.y, 3, d.J[0], d.J[1], d.J[2], d.Jf[0], d.Jf[1], d.Jf[2]);
}

template <typename R>
__global__ __launch_bounds__(NT) void k_yee(SimDev<R> d)
{
    yee_body(d, xcd_remap(blockIdx.x, gridDim.x));
}

// A Yee launch is short, so its blocks' completion counts would pile up on one
// address; the step end runs as a one-block launch instead.  When a push of
// the step asked for it (DevState::relay), the block then lays out the
// particle segments of every species anew for the next push.
template <typename R>
__global__ __launch_bounds__(NTO) void k_step_end(SimDev<R> d)
{
    const bool relay = glob<const DevState>(d.st)->relay != 0;
    if (threadIdx.x == 0) step_end_body(d);
    if (!relay) return;  // block-uniform
    __syncthreads();     // the layouts read the new window origin
    layouts_body(d);
    if (threadIdx.x == 0) d.st->relay = 0;
}

template <typename R>
__global__ __launch_bounds__(NT) void k_yee_b(const SimDev<R> *__restrict__ ds,
                                             const BatchDev *__restrict__ b)
{
    int2 it;
    if (batch_item(b, &it)) yee_body(ds[it.x], it.y);
}

// The batch's step end: one thread per simulation, then the relayouts that
// pushes asked for, one simulation after another (most steps ask for none).
template <typename R>
__global__ __launch_bounds__(NTO) void k_step_end_b(const SimDev<R> *__restrict__ ds,
                                                    const BatchDev *__restrict__ b)
{
    __shared__ int s_n;
    __shared__ int s_list[NTO];
    const int n = b->nsim;
    for (int i0 = 0; i0 < n; i0 += NTO) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        const int i = i0 + (int)threadIdx.x;
        if (i < n) {
            if (glob<const DevState>(ds[i].st)->relay) s_list[atomicAdd(&s_n, 1)] = i;
            step_end_body(ds[i]);
        }
        __syncthreads();
        const int m = s_n;
        for (int k = 0; k < m; ++k) {
            const SimDev<R> &d = ds[s_list[k]];
            layouts_body(d);
            if (threadIdx.x == 0) d.st->relay = 0;
        }
        __syncthreads();  // s_n and s_list are reused
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename R>
hipError_t Launch<R>::push_deposit(const SimDev<R> &d, hipStream_t s)
{
    if (d.direct) {
        hipLaunchKernelGGL(k_zero_j<R>, dim3(512), dim3(NT), 0, s, d);
        hipError_t e = hipGetLastError();
        for (int colour = 0; colour < 4 && e == hipSuccess; ++colour) {
            hipLaunchKernelGGL(k_push_colour<R>, dim3(d.ntiles / 4), dim3(NTP), 0, s, d, colour);
            e = hipGetLastError();
        }
        return e;
    }
    const dim3 grid(d.ntiles * d.nsb);
    if (d.push_bt == NTP_BIG)
        hipLaunchKernelGGL((k_push_deposit<R, NTP_BIG>), grid, dim3(NTP_BIG), 0, s, d);
    else
        hipLaunchKernelGGL((k_push_deposit<R, NTP>), grid, dim3(NTP), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::order(const SimDev<R> &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_order<R>, dim3(d.nsp + 1), dim3(NTO), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::layout_b(const SimDev<R> *ds, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_layout_b<R>, dim3(n), dim3(NTO), 0, s, ds);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::settle(const SimDev<R> &d, hipStream_t s, bool only_if_shift,
                             bool unpend)
{
    if (d.nsp > 0) {
        hipLaunchKernelGGL(k_settle<R>, dim3(d.ntiles), dim3(MT), 0, s, d, (int)only_if_shift);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!unpend) return hipSuccess;
    hipLaunchKernelGGL(k_unpend<R>, dim3(1), dim3(64), 0, s, d, (int)only_if_shift);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::fold(const SimDev<R> &d, int nplanes, R *o0, R *o1, R *o2, hipStream_t s)
{
    if (nplanes == 3) {
        const dim3 grid(fold_units(d.ntx, d.nty));
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(64), 0, s, d, o0, o1, o2); };
        static_assert(MAX_SP == 4, "one instance per species-block count");
        switch (d.nsb) {
        case 1: go(k_fold_s<R, 1>); break;
        case 2: go(k_fold_s<R, 2>); break;
        case 3: go(k_fold_s<R, 3>); break;
        default: go(k_fold_s<R, 4>); break;
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_fold<R>, dim3(d.ntiles), dim3(NT), 0, s, d, nplanes, o0, o1, o2);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::filter(const SimDev<R> &d, int nplanes, const R *i0, const R *i1,
                             const R *i2, R *o0, R *o1, R *o2, hipStream_t s, bool before_shift)
{
    const int rf = d.npass + (d.compensate ? 1 : 0);
    if (nplanes == 3 && rf >= 1 && rf <= MAX_FR) {
        const int nst = (d.ny + FS_S - 1) / FS_S;
        auto go = [&](auto kern, int w) {
            hipLaunchKernelGGL(kern, dim3(((d.nxs + w - 1) / w) * nst), dim3(64), 0, s, d, i0, i1,
                               i2, o0, o1, o2, (int)before_shift);
        };
        static_assert(MAX_FR == 4, "one instance per filter halo");
        switch (rf) {
        case 1: go(k_filter_s<R, 1>, 62); break;
        case 2: go(k_filter_s<R, 2>, 60); break;
        case 3: go(k_filter_s<R, 3>, 58); break;
        default: go(k_filter_s<R, 4>, 56); break;
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_filter<R>, dim3(d.ntiles), dim3(NT), 0, s, d, nplanes, i0, i1, i2, o0,
                       o1, o2);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::yee(const SimDev<R> &d, hipStream_t s)
{
    const int rf = d.npass > 0 ? d.npass + (d.compensate ? 1 : 0) : 0;
    const dim3 grid(yee_units(d.nxs, d.ny, rf));
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(64), 0, s, d); };
    static_assert(MAX_FR == 4, "one instance per filter halo");
    if (folds_in_yee(d)) {  // filter halo 0 or 1
        if (rf == 0)
            go(k_fold_yee_s<R, 0>);
        else
            go(k_fold_yee_s<R, 1>);
    } else {
        switch (rf) {
        case 0: go(k_yee_s<R, 0>); break;
        case 1: go(k_yee_s<R, 1>); break;
        case 2: go(k_yee_s<R, 2>); break;
        case 3: go(k_yee_s<R, 3>); break;
        default: go(k_yee_s<R, 4>); break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_step_end<R>, dim3(1), dim3(NTO), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::window(const SimDev<R> &d, hipStream_t s)
{
    if (d.nx >= TX) {
        hipLaunchKernelGGL(k_window<R>, dim3(2 * d.nty * d.nsp + 1), dim3(NT), 0, s, d);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_unpend<R>, dim3(1), dim3(64), 0, s, d, 1);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(k_window_clear<R>, dim3(d.nty * d.nsp + 1), dim3(NT), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || d.nsp == 0) return e;
    hipLaunchKernelGGL(k_window_inject<R>, dim3(d.nty * d.nsp), dim3(NT), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::load(const SimDev<R> &d, int sp, hipStream_t s)
{
    hipLaunchKernelGGL(k_load<R>, dim3(d.ntiles), dim3(NT), 0, s, d, sp);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::rho(const SimDev<R> &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rho<R>, dim3(d.ntiles), dim3(NT), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::g0(const SimDev<R> &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_g0<R>, dim3(NB_DIAG), dim3(NT), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::diag(const SimDev<R> &d, int has_prev, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_grid<R>, dim3(NB_DIAG), dim3(NT), 0, s, d, has_prev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_ke<R>, dim3(d.ntiles), dim3(NT), 0, s, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final<R>, dim3(1), dim3(NT), 0, s, d);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::copy_plane(const R *src, R *dst, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy<R>, dim3(NB_DIAG), dim3(NT), 0, s, src, dst, n);
    return hipGetLastError();
}

// One step of a batch: grid = the work-list capacity the graph was captured
// for; `ds` and `b` live in device memory.
template <typename R>
hipError_t launch_batch_step(const SimDev<R> *ds, const BatchDev *b, int grid, hipStream_t s,
                             int rf, int grid_fold, int grid_yee)
{
    hipLaunchKernelGGL(k_push_deposit_b<R>, dim3(grid), dim3(NTB), 0, s, ds, b);
    if (rf >= 0 && rf <= MAX_FR) {
        // the streaming forms, when every simulation has the same filter halo
        hipLaunchKernelGGL(k_fold_sb<R>, dim3(grid_fold), dim3(64), 0, s, ds, b);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid_yee), dim3(64), 0, s, ds, b);
        };
        static_assert(MAX_FR == 4, "one instance per filter halo");
        switch (rf) {
        case 0: go(k_yee_sb<R, 0>); break;
        case 1: go(k_yee_sb<R, 1>); break;
        case 2: go(k_yee_sb<R, 2>); break;
        case 3: go(k_yee_sb<R, 3>); break;
        default: go(k_yee_sb<R, 4>); break;
        }
    } else {
        hipLaunchKernelGGL(k_fold_b<R>, dim3(grid), dim3(NT), 0, s, ds, b);
        hipLaunchKernelGGL(k_filter_b<R>, dim3(grid), dim3(NT), 0, s, ds, b);
        hipLaunchKernelGGL(k_yee_b<R>, dim3(grid), dim3(NT), 0, s, ds, b);
    }
    hipLaunchKernelGGL(k_step_end_b<R>, dim3(1), dim3(NTO), 0, s, ds, b);
    return hipGetLastError();
}

template hipError_t launch_batch_step<float>(const SimDev<float> *, const BatchDev *, int,
                                             hipStream_t, int, int, int);
template hipError_t launch_batch_step<double>(const SimDev<double> *, const BatchDev *, int,
                                              hipStream_t, int, int, int);

template struct Launch<float>;
template struct Launch<double>;

}  // namespace pic
