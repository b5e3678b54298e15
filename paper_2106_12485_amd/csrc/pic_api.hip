// Host side of libpic: the C ABI declared in include/pic.h.  Validates the
// configuration, lays the simulation out in the caller's device arena, moves
// host state in and out, and enqueues the kernels of pic_kernels.hip on the
// caller's stream (directly, or from captured HIP graphs of one or eight steps).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "pic.h"
#include "pic_dev.h"

using namespace pic;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// No C++ exception crosses the ABI: a failed host allocation (or a request
// for more than a vector can hold) becomes PIC_E_NOMEM, anything else
// PIC_E_STATE, with the message in pic_last_error.  Entry points returning a
// status (int, long long) return that code; those returning a size return 0.
template <typename T, typename F>
T guarded(F &&body) noexcept
{
    int code = PIC_E_STATE;
    try {
        return body();
    } catch (const std::bad_alloc &) {
        code = fail(PIC_E_NOMEM, "host memory allocation failed");
    } catch (const std::length_error &) {
        code = fail(PIC_E_NOMEM, "host buffer larger than a vector can hold");
    } catch (const std::exception &e) {
        code = fail(PIC_E_STATE, std::string("C++ exception: ") + e.what());
    } catch (...) {
        code = fail(PIC_E_STATE, "unknown C++ exception");
    }
    return std::is_signed<T>::value ? (T)code : T(0);
}

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(PIC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Arena layout of one simulation.
struct Layout {
    int nxs, ntx, nty, ntiles;
    long long pool[MAX_SP];  // particle slots per buffer
    int maxseg[MAX_SP];  // most slots of one tile's segment
    int cap_out;
    int push_bt, nsb;  // threads per push block; push blocks per tile
    size_t rs;  // bytes of the working precision
    size_t plane;  // elements of one storage plane
    size_t off_state, off_F, off_J, off_Jf, off_rho, off_rho_f, off_rho_prev, off_g0, off_blk,
        off_red, off_res, off_order;
    size_t off_sp[MAX_SP];  // start of each species block
    size_t sp_bytes[MAX_SP];
    size_t total;
};

// Particles the loader puts in each tile for species s (window origin 0, no
// shift): per storage column, the sub-positions m whose lab-frame x, in
// double exactly as k_load evaluates it, lies in [x_lo, x_hi), times ppc_y
// and the tile's rows.  Empty without a load or density.
std::vector<long long> load_counts(const pic_cfg *c, int nxs, int ntx, int nty, int s)
{
    std::vector<long long> cnt((size_t)ntx * nty, 0);
    const pic_species_cfg &p = c->sp[s];
    if (!c->load || !(p.density > 0.0)) return cnt;
    const double dx = c->lx / c->nx;
    std::vector<long long> col((size_t)nxs, 0);
    for (int gx = 0; gx < c->nx; ++gx) {
        int m_in = 0;
        for (int m = 0; m < p.ppc_x; ++m) {
            const double xo = ((double)m + 0.5) / (double)p.ppc_x;
            const double xlab = ((double)gx + xo) * dx;
            m_in += xlab >= p.x_lo && xlab < p.x_hi;
        }
        col[gx] = (long long)m_in * p.ppc_y;
    }
    for (int ty = 0; ty < nty; ++ty) {
        const int h = std::min(TY, c->ny - ty * TY);
        for (int tx = 0; tx < ntx; ++tx) {
            long long n = 0;
            for (int gx = tx * TX; gx < std::min(nxs, tx * TX + TX); ++gx) n += col[gx];
            cnt[(size_t)tx + (size_t)ty * ntx] = n * h;
        }
    }
    return cnt;
}

// Segments from per-tile counts (the host's form of the device relayout,
// with no outflow known yet): each tile its count (+ extra, if given)
// rounded up to 64 slots, plus a share of the rest of the pool in
// proportion to count + average count, at most maxseg, in tile order.
// False if the counts do not fit.
bool layout_from_counts(const std::vector<long long> &cnt, long long pool, long long maxseg,
                        std::vector<long long> *start, std::vector<int> *seg,
                        const std::vector<long long> *extra = nullptr)
{
    const size_t n = cnt.size();
    long long total = 0, need = 0;
    auto want = [&](size_t t) {
        const long long v = cnt[t] + (extra ? (*extra)[t] : 0);
        return std::min(maxseg, (v + 63) / 64 * 64);
    };
    for (size_t t = 0; t < n; ++t) {
        if (cnt[t] > maxseg) return false;
        total += cnt[t];
        need += want(t);
    }
    const long long spare = pool - need;
    if (spare < 0) return false;
    const double avg = n ? (double)total / (double)n : 0.0;
    const double wsum = (double)total + avg * (double)n;
    start->assign(n, 0);
    seg->assign(n, 0);
    long long at = 0;
    for (size_t t = 0; t < n; ++t) {
        const long long base = want(t);
        const long long share =
            wsum > 0 ? (long long)((double)spare * ((double)cnt[t] + avg) / wsum) / 64 * 64 : 0;
        const long long cap = std::min(maxseg, base + share);
        (*start)[t] = at;
        (*seg)[t] = (int)cap;
        at += cap;
    }
    return true;
}

int layout(const pic_cfg *c, Layout *L)
{
    if (!c) return fail(PIC_E_ARG, "cfg is NULL");
    // cell indices are packed in 16 bits per axis (storage columns with the
    // moving window: nx plus the gap, rounded up to the tile width)
    if (c->nx < 2 || c->ny < 2 || c->nx > 65535 || c->ny > 65535)
        return fail(PIC_E_ARG, "nx and ny must be in [2, 65535]");
    if (c->moving_window && (c->nx + TX + 2 + TX - 1) / TX * TX > 65536)
        return fail(PIC_E_ARG, "with the moving window nx must be at most 65518 (the storage "
                               "width adds an 18-cell gap, rounded to the tile width)");
    if (!(c->lx > 0) || !(c->ly > 0) || !(c->dt > 0))
        return fail(PIC_E_ARG, "lx, ly and dt must be positive");
    if (c->n_species < 0 || c->n_species > PIC_MAX_SPECIES)
        return fail(PIC_E_ARG, "n_species must be in [0, 4]");
    if (c->filter_passes < 0 || c->filter_passes + (c->filter_compensate ? 1 : 0) > MAX_FR ||
        (c->filter_compensate && c->filter_passes == 0))
        return fail(PIC_E_ARG, "filter: passes in [0, 4], compensator needs passes >= 1, "
                               "passes + compensator <= 4");
    const double dx = c->lx / c->nx, dy = c->ly / c->ny;
    if (!(c->dt * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy)) < 1.0))
        return fail(PIC_E_CFL, "dt violates the Courant limit dt < 1/sqrt(1/dx^2 + 1/dy^2)");
    const double cf = c->capacity_factor > 0 ? c->capacity_factor : 2.0;
    for (int s = 0; s < c->n_species; ++s) {
        const pic_species_cfg &p = c->sp[s];
        if (p.ppc_x < 1 || p.ppc_y < 1 || p.ppc_x * p.ppc_y > 1024)
            return fail(PIC_E_ARG, "ppc_x, ppc_y must be >= 1 with ppc_x*ppc_y <= 1024");
        if (p.q_over_m == 0.0 || !std::isfinite(p.q_over_m))
            return fail(PIC_E_ARG, "q_over_m must be finite and non-zero");
        if (p.density < 0) return fail(PIC_E_ARG, "density must be >= 0");
    }
    L->nxs = c->moving_window ? ((c->nx + TX + 2 + TX - 1) / TX) * TX : c->nx;
    L->ntx = (L->nxs + TX - 1) / TX;
    L->nty = (c->ny + TY - 1) / TY;
    if (c->deposit_mode != 0 && c->deposit_mode != 1)
        return fail(PIC_E_ARG, "deposit_mode must be 0 (reduction) or 1 (commutative)");
    if (c->deposit_mode == 1 && (c->moving_window || (L->ntx & 1) || (L->nty & 1)))
        return fail(PIC_E_ARG, "the commutative deposit needs a periodic box with an even "
                               "number of 16-cell tiles along each axis");
    // A tile block reaches one cell below and two above its tile.  Same-colour
    // tiles are two tiles apart, with one tile of width w between them (or the
    // last tile, across the periodic seam), so their blocks are disjoint only
    // if that tile is at least 3 cells wide: every middle tile is 16 wide, the
    // last one n % 16.
    if (c->deposit_mode == 1 && (L->nxs % TX == 1 || L->nxs % TX == 2 || c->ny % TY == 1 ||
                                 c->ny % TY == 2))
        return fail(PIC_E_ARG, "the commutative deposit needs the last tile along each axis "
                               "to be at least 3 cells wide (n % 16 not 1 or 2)");
    L->ntiles = L->ntx * L->nty;
    L->rs = c->fp64 ? 8 : 4;
    L->plane = (size_t)L->nxs * c->ny;
    // Particle slots per buffer and species: capacity_factor times the most
    // particles the species can hold: its initial load on a periodic box
    // (the count is then conserved), or the whole box at its ppc with the
    // moving window (which loads plasma as it moves) or without a load (room
    // for particles set from the host); plus 64 slots per tile for rounding.
    // A tile's segment holds at most 8 times a full tile at the species' ppc
    // (this bounds the fixed-point scale of the current sums).
    long long full_tile = 0;  // largest full-tile load over the species
    for (int s = 0; s < c->n_species; ++s) {
        const pic_species_cfg &p = c->sp[s];
        const long long ppc = (long long)p.ppc_x * p.ppc_y;
        long long nmax = (long long)c->nx * c->ny * ppc;
        if (!c->moving_window && c->load && p.density > 0.0) {
            long long n0 = 0;
            for (long long v : load_counts(c, L->nxs, L->ntx, L->nty, s)) n0 += v;
            nmax = n0;
        }
        // with the moving window, also room for the columns the next 16
        // steps load at the right edge (a layout reserves it ahead)
        const double inj = c->moving_window && p.density > 0.0 ? 16.0 * c->ny * ppc : 0.0;
        const double want = cf * (double)nmax + inj + 64.0 * L->ntiles;
        if (want > (double)(1LL << 40)) return fail(PIC_E_ARG, "capacity_factor too large");
        L->pool[s] = ((long long)std::ceil(want) + 63) / 64 * 64;
        L->maxseg[s] = (int)std::min<long long>(L->pool[s], 8 * ppc * TX * TY);
        full_tile = std::max(full_tile, ppc * TX * TY);
    }
    // Outbox: a quarter of a full tile's load.  A particle crosses at most
    // one cell per step, so only those in the tile's outer ring of cells (60
    // of 256) can leave: a uniformly filled tile sends at most 23% of its
    // particles, even when every one of them moves outwards at close to c.
    L->cap_out = (int)std::max<long long>(256, (full_tile / 4 + 63) / 64 * 64);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L->off_state = take(sizeof(DevState));
    L->off_F = take(12 * L->plane * L->rs);
    L->off_J = take(3 * L->plane * L->rs);
    L->off_Jf = take(3 * L->plane * L->rs);
    L->off_rho = take(L->plane * L->rs);
    L->off_rho_f = take(L->plane * L->rs);
    L->off_rho_prev = take(L->plane * L->rs);
    L->off_g0 = take(L->plane * 8);
    // Tiles loaded with BIG_TILE particles or more take 1024-thread push
    // blocks and, with several species, one block per species, each leaving
    // its current as exact 64-bit sums (see push_body).
    long long per_tile = 0;
    for (int s = 0; s < c->n_species; ++s)
        per_tile += (long long)c->sp[s].ppc_x * c->sp[s].ppc_y * TX * TY;
    L->push_bt = per_tile >= BIG_TILE ? NTP_BIG : NTP;
    L->nsb = per_tile >= BIG_TILE && c->deposit_mode == 0 && c->n_species > 1 ? c->n_species : 1;
    L->off_blk = take((size_t)L->ntiles * 3 * BP * (L->nsb > 1 ? L->nsb * 8 : L->rs));
    L->off_red = take(((size_t)NB_DIAG * 5 + (size_t)L->ntiles * MAX_SP) * 8);
    L->off_res = take(N_RED * 8);
    L->off_order = take((size_t)L->ntiles * L->nsb * 4);
    const size_t obs = (size_t)L->ntiles * L->cap_out;
    for (int s = 0; s < c->n_species; ++s) {
        const size_t slots = (size_t)L->pool[s];
        size_t b = 0;
        // two particle buffers (packed cell + 5 components + per-tile count,
        // segment start and segment slots)
        b += 2 * (align256(slots * 4) + 5 * align256(slots * L->rs) +
                  2 * align256((size_t)L->ntiles * 4) + align256((size_t)L->ntiles * 8));
        // each tile's count at the last layout check, its need there, and
        // its last inflow
        b += 3 * align256((size_t)L->ntiles * 4);
        // two outboxes (cell, direction byte, 5 components, per-tile count)
        b += 2 * (align256(obs * 4) + align256(obs) + 5 * align256(obs * L->rs) +
                  align256((size_t)L->ntiles * 4));
        L->off_sp[s] = take(b);
        L->sp_bytes[s] = b;
    }
    L->total = o;
    return PIC_OK;
}

// Fill the device descriptor with arena pointers.
template <typename R>
void describe(const pic_cfg *c, const Layout &L, char *a, SimDev<R> *d)
{
    std::memset((void *)d, 0, sizeof(*d));
    d->nx = c->nx;
    d->ny = c->ny;
    d->nxs = L.nxs;
    d->ntx = L.ntx;
    d->nty = L.nty;
    d->rx = fold_reach(L.nxs, TX);
    d->ry = fold_reach(c->ny, TY);
    d->ntiles = L.ntiles;
    d->window = c->moving_window ? 1 : 0;
    d->nsp = c->n_species;
    d->cap_out = L.cap_out;
    d->npass = c->filter_passes;
    d->compensate = c->filter_compensate ? 1 : 0;
    d->direct = c->deposit_mode == 1 ? 1 : 0;
    d->push_bt = L.push_bt;
    d->nsb = L.nsb;
    d->dx_d = c->lx / c->nx;
    d->dy_d = c->ly / c->ny;
    d->dt_d = c->dt;
    d->dx = (R)d->dx_d;
    d->dy = (R)d->dy_d;
    d->dt = (R)d->dt_d;
    d->idx = (R)(1.0 / d->dx_d);
    d->idy = (R)(1.0 / d->dy_d);
    d->dt_dx = (R)(d->dt_d / d->dx_d);
    d->dt_dy = (R)(d->dt_d / d->dy_d);
    d->jxs = (R)(d->dx_d / d->dt_d);
    d->jys = (R)(d->dy_d / d->dt_d);
    // Fixed-point scale 2^-e of the LDS sums.  The terms one particle adds to
    // one LDS entry over its step total at most |q_p| (|v| < 1; weights and
    // path fractions <= 1).  A push block takes its tile's particles and the
    // arrivals of the last hand-off; unless it flags a capacity error, those
    // that stay fit the tile's segment (at most maxseg slots) and those that
    // leave fit the outbox, so an entry never exceeds the sum of |q_p| over
    // maxseg + outbox slots of every species.  Take the largest e that keeps
    // that bound below 2^62.
    double bound = 0.0;
    for (int s = 0; s < c->n_species; ++s) {
        const pic_species_cfg &p = c->sp[s];
        bound += (double)(L.maxseg[s] + L.cap_out) * p.density / (p.ppc_x * p.ppc_y);
    }
    const int e = bound > 0 ? std::min(120, 62 - (int)std::ceil(std::log2(bound))) : 60;
    d->jq = (R)std::ldexp(1.0, sizeof(R) == 4 ? e - 32 : e);
    d->jq_inv = std::ldexp(1.0, -e);
    d->key0 = (unsigned)(c->seed & 0xffffffffull);
    d->key1 = (unsigned)(c->seed >> 32);
    R *F = (R *)(a + L.off_F);
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 6; ++k) d->F[b][k] = F + (size_t)(b * 6 + k) * L.plane;
    for (int k = 0; k < 3; ++k) {
        d->J[k] = (R *)(a + L.off_J) + (size_t)k * L.plane;
        d->Jf[k] = c->filter_passes > 0 ? (R *)(a + L.off_Jf) + (size_t)k * L.plane : d->J[k];
    }
    d->rho = (R *)(a + L.off_rho);
    d->rho_f = (R *)(a + L.off_rho_f);
    d->rho_prev = (R *)(a + L.off_rho_prev);
    d->g0 = (double *)(a + L.off_g0);
    d->blk = (R *)(a + L.off_blk);
    d->order = (int *)(a + L.off_order);
    d->red = (double *)(a + L.off_red);
    d->res = (double *)(a + L.off_res);
    d->st = (DevState *)(a + L.off_state);
    for (int s = 0; s < c->n_species; ++s) {
        const pic_species_cfg &p = c->sp[s];
        SpDev<R> &P = d->sp[s];
        const size_t slots = (size_t)L.pool[s];
        const size_t obs = (size_t)L.ntiles * L.cap_out;
        char *q = a + L.off_sp[s];
        auto next = [&](size_t bytes) {
            char *r = q;
            q += align256(bytes);
            return r;
        };
        for (int b = 0; b < 2; ++b) {
            PartBuf<R> &B = P.pb[b];
            B.cell = (int *)next(slots * 4);
            B.x = (R *)next(slots * L.rs);
            B.y = (R *)next(slots * L.rs);
            B.ux = (R *)next(slots * L.rs);
            B.uy = (R *)next(slots * L.rs);
            B.uz = (R *)next(slots * L.rs);
            B.count = (int *)next((size_t)L.ntiles * 4);
            P.start[b] = (long long *)next((size_t)L.ntiles * 8);
            P.seg[b] = (int *)next((size_t)L.ntiles * 4);
        }
        P.snap = (int *)next((size_t)L.ntiles * 4);
        P.need = (int *)next((size_t)L.ntiles * 4);
        P.inflow = (int *)next((size_t)L.ntiles * 4);
        for (int b = 0; b < 2; ++b) {
            P.ob_cell[b] = (int *)next(obs * 4);
            P.ob_dir[b] = (unsigned char *)next(obs);
            P.ob_x[b] = (R *)next(obs * L.rs);
            P.ob_y[b] = (R *)next(obs * L.rs);
            P.ob_ux[b] = (R *)next(obs * L.rs);
            P.ob_uy[b] = (R *)next(obs * L.rs);
            P.ob_uz[b] = (R *)next(obs * L.rs);
            P.ob_count[b] = (int *)next((size_t)L.ntiles * 4);
        }
        const double qp = (p.q_over_m < 0 ? -1.0 : 1.0) * p.density / (p.ppc_x * p.ppc_y);
        P.qm = (R)p.q_over_m;
        P.qp = (R)qp;
        P.tau = (R)(0.5 * c->dt * p.q_over_m);
        P.pool = L.pool[s];
        P.maxseg = L.maxseg[s];
        P.ppc_x = p.ppc_x;
        P.ppc_y = p.ppc_y;
        P.density = p.density;
        P.x_lo = p.x_lo;
        P.x_hi = p.x_hi;
        for (int k = 0; k < 3; ++k) {
            P.uth[k] = p.uth[k];
            P.ufl[k] = p.ufl[k];
        }
    }
}

// The initial laser of pic_laser_cfg at (x, y) (lab frame, t = 0).
double laser_eperp(const pic_laser_cfg &l, double x, double y)
{
    const double d = x - l.x_center;
    if (std::fabs(d) > 2.0 * l.fwhm) return 0.0;
    const double g = std::exp(-2.0 * std::log(2.0) * d * d / (l.fwhm * l.fwhm));
    const double z = x - l.focus, r = y - l.axis;
    const double zr = 0.5 * l.omega0 * l.W0 * l.W0;
    const double wz = l.W0 * std::sqrt(1.0 + (z / zr) * (z / zr));
    const double curv = (z == 0.0) ? 0.0 : l.omega0 * r * r * z / (2.0 * (z * z + zr * zr));
    return l.a0 * l.omega0 * g * std::sqrt(l.W0 / wz) * std::exp(-(r * r) / (wz * wz)) *
           std::cos(l.omega0 * d + curv - 0.5 * std::atan(z / zr));
}

}  // namespace

// Pushes between two work-order launches (each also checks the particle
// layout): the first step of every 8-step graph, and before a push that
// follows 8 others without one.
constexpr int GRAPH_STEPS_N = 8;

struct pic_sim {
    pic_cfg cfg;
    Layout L;
    char *arena;
    SimDev<float> df;
    SimDev<double> dd;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;   // one step
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec_n = nullptr; // GRAPH_STEPS steps
    hipGraph_t graph_n = nullptr;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    int ev_used = 0;
    double ms[PIC_NK];
    long long launches[PIC_NK];
    // diagnostics
    long long rho_prev_iter = -2;
    int since_order = GRAPH_STEPS_N;  // pushes enqueued since the last work order
                                      // and layout check (at most GRAPH_STEPS)
    DevState hs;  // host copy, valid after read_state
    unsigned long long uid = 0;  // unique per pic_init (handles may reuse addresses)
};

namespace {
std::atomic<unsigned long long> g_next_uid{1};
}

namespace {

int read_state(pic_sim *s, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(&s->hs, s->arena + s->L.off_state, sizeof(DevState),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PIC_OK;
}

int write_state(pic_sim *s, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(s->arena + s->L.off_state, &s->hs, sizeof(DevState),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return PIC_OK;
}

// Flush recorded event pairs into the per-kernel sums.
int timing_flush(pic_sim *s)
{
    for (int i = 0; i < s->ev_used; ++i) {
        HIPCHK(hipEventSynchronize(s->ev[2 * i + 1]));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->ms[s->ev_kind[i]] += ms;
        s->launches[s->ev_kind[i]] += 1;
    }
    s->ev_used = 0;
    return PIC_OK;
}

// Run `fn` (which enqueues one kernel class), bracketed by events if timing.
template <typename Fn>
int timed(pic_sim *s, int kind, hipStream_t st, Fn fn)
{
    if (!s->timing) {
        hipError_t e = fn();
        if (e != hipSuccess) return fail(PIC_E_HIP, std::string("launch: ") + hipGetErrorString(e));
        return PIC_OK;
    }
    if (s->ev_used >= 4096) {
        int rc = timing_flush(s);
        if (rc) return rc;
    }
    while ((int)s->ev.size() < 2 * (s->ev_used + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        s->ev.push_back(e);
    }
    if ((int)s->ev_kind.size() < s->ev_used + 1) s->ev_kind.resize(s->ev_used + 1);
    HIPCHK(hipEventRecord(s->ev[2 * s->ev_used], st));
    hipError_t e = fn();
    if (e != hipSuccess) return fail(PIC_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    HIPCHK(hipEventRecord(s->ev[2 * s->ev_used + 1], st));
    s->ev_kind[s->ev_used] = kind;
    s->ev_used += 1;
    return PIC_OK;
}

// Append pending leavers to their tiles (no-op when none are pending).
template <typename R>
int enqueue_settle(pic_sim *s, const SimDev<R> &d, hipStream_t st, bool only_if_shift = false,
                   bool unpend = true)
{
    return timed(s, 1, st, [&] { return Launch<R>::settle(d, st, only_if_shift, unpend); });
}

// The push's work order (heaviest tiles first) and the particle layout are
// rewritten at most every GRAPH_STEPS pushes: particle counts move slowly,
// and the order only has to be close.
constexpr int GRAPH_STEPS = GRAPH_STEPS_N;

// The push of one step, preceded by a new work order when `order` is set.
template <typename R>
int enqueue_push(pic_sim *s, const SimDev<R> &d, hipStream_t st, bool order)
{
    if (order) {  // the colour-phased pushes take no order, but need the layouts
        const int rc = timed(s, 6, st, [&] { return Launch<R>::order(d, st); });
        if (rc) return rc;
    }
    return timed(s, 0, st, [&] { return Launch<R>::push_deposit(d, st); });
}

// a push launched directly (not from a graph): a new order after
// GRAPH_STEPS pushes without one
template <typename R>
int enqueue_push_direct(pic_sim *s, const SimDev<R> &d, hipStream_t st)
{
    const bool order = s->since_order >= GRAPH_STEPS;
    s->since_order = order ? 1 : s->since_order + 1;
    return enqueue_push(s, d, st, order);
}

// a1-a4: push + deposit; the leavers are then appended to their new tiles
template <typename R>
int enqueue_deposit(pic_sim *s, const SimDev<R> &d, hipStream_t st)
{
    int rc = enqueue_push_direct(s, d, st);
    if (rc) return rc;
    return enqueue_settle(s, d, st);
}

// a5-a8.  The window kernels need complete tiles, so leavers are settled
// first with the moving window.
template <typename R>
int enqueue_field_advance(pic_sim *s, const SimDev<R> &d, hipStream_t st)
{
    int rc = PIC_OK;
    if (!d.direct && !folds_in_yee(d)) {
        rc = timed(s, 2, st, [&] { return Launch<R>::fold(d, 3, d.J[0], d.J[1], d.J[2], st); });
        if (rc) return rc;
    }
    // the Yee launch filters J itself (Jf is only written on request), and
    // folds it first where folds_in_yee
    rc = timed(s, 4, st, [&] { return Launch<R>::yee(d, st); });
    if (rc) return rc;
    if (d.window) {
        // the column shift needs every particle in its tile; without a shift
        // the next push takes the pending leavers from the outboxes itself.
        // The window launch clears the pending flag after a settle.
        rc = enqueue_settle(s, d, st, true, false);
        if (rc) return rc;
        rc = timed(s, 5, st, [&] { return Launch<R>::window(d, st); });
    }
    return rc;
}

// One step of pic_step: the next push takes the pending leavers directly
// from the outboxes, so no hand-off launch is needed between steps.
template <typename R>
int enqueue_step(pic_sim *s, const SimDev<R> &d, hipStream_t st, bool order)
{
    int rc = enqueue_push(s, d, st, order);
    if (rc) return rc;
    return enqueue_field_advance(s, d, st);
}

// Charge density of the current particles: rho, and F rho in rho_f.
template <typename R>
int enqueue_rho(const SimDev<R> &d, hipStream_t st)
{
    HIPCHK(Launch<R>::rho(d, st));
    HIPCHK(Launch<R>::fold(d, 1, d.rho, nullptr, nullptr, st));
    if (d.npass > 0)
        HIPCHK(Launch<R>::filter(d, 1, d.rho, nullptr, nullptr, d.rho_f, nullptr, nullptr, st));
    else
        HIPCHK(Launch<R>::copy_plane(d.rho, d.rho_f, (long long)d.nxs * d.ny, st));
    return PIC_OK;
}

template <typename R>
int gauss_baseline(pic_sim *s, const SimDev<R> &d, hipStream_t st)
{
    int rc = enqueue_rho(d, st);
    if (rc) return rc;
    HIPCHK(Launch<R>::g0(d, st));
    HIPCHK(hipStreamSynchronize(st));
    s->rho_prev_iter = -2;
    return PIC_OK;
}

// With the moving window, the room per tile for the columns the next 16
// steps load at the right edge (storage columns origin + nx .. + 15, at most
// one per step); zero otherwise.
std::vector<long long> window_room(const pic_cfg &c, const Layout &L, int sp, int origin)
{
    std::vector<long long> extra((size_t)L.ntiles, 0);
    const pic_species_cfg &p = c.sp[sp];
    if (!c.moving_window || !(p.density > 0.0)) return extra;
    for (int k = 0; k < 16; ++k) {
        const int gx = (origin + c.nx + k) % L.nxs;
        for (int ty = 0; ty < L.nty; ++ty)
            extra[(size_t)(gx / TX) + (size_t)ty * L.ntx] +=
                (long long)std::min(TY, c.ny - ty * TY) * p.ppc_x * p.ppc_y;
    }
    return extra;
}

// Upload a species' segments to both buffers' layout arrays, and the
// counts they were made for as the growth snapshot (synchronises: the host
// vectors are freed on return).
template <typename R>
int upload_layout(const SpDev<R> &P, const std::vector<long long> &start,
                  const std::vector<int> &seg, const std::vector<int> &snap, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(P.snap, snap.data(), snap.size() * 4, hipMemcpyHostToDevice, st));
    for (int b = 0; b < 2; ++b) {
        HIPCHK(hipMemcpyAsync(P.start[b], start.data(), start.size() * 8, hipMemcpyHostToDevice,
                              st));
        HIPCHK(hipMemcpyAsync(P.seg[b], seg.data(), seg.size() * 4, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return PIC_OK;
}

template <typename R>
int do_init(pic_sim *s, const SimDev<R> &d, hipStream_t st)
{
    const pic_cfg &c = s->cfg;
    const Layout &L = s->L;
    HIPCHK(hipMemsetAsync(s->arena, 0, L.total, st));
    {
        // the push's first work order: every item once (the field launch of
        // each step rewrites it, heaviest first)
        std::vector<int> ord((size_t)L.ntiles * L.nsb);
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
        HIPCHK(hipMemcpyAsync(d.order, ord.data(), ord.size() * sizeof(int),
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (c.laser.on) {
        std::vector<R> h(L.plane * 6, R(0));
        const pic_laser_cfg &l = c.laser;
        const double cp = std::cos(l.pol_angle), sn = std::sin(l.pol_angle);
        const double dx = d.dx_d, dy = d.dy_d;
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t g = (size_t)i + (size_t)j * L.nxs;  // origin 0 at init
                const double xi = i * dx, xh = (i + 0.5) * dx, yj = j * dy, yh = (j + 0.5) * dy;
                h[1 * L.plane + g] = (R)(cp * laser_eperp(l, xi, yh));   // Ey (i, j+1/2)
                h[2 * L.plane + g] = (R)(sn * laser_eperp(l, xi, yj));   // Ez (i, j)
                h[4 * L.plane + g] = (R)(-sn * laser_eperp(l, xh, yj));  // By (i+1/2, j)
                h[5 * L.plane + g] = (R)(cp * laser_eperp(l, xh, yh));   // Bz (i+1/2, j+1/2)
            }
        HIPCHK(hipMemcpyAsync(d.F[0][0], h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice,
                              st));
        HIPCHK(hipStreamSynchronize(st));
    }
    // segments of every tile from the load's counts, the same in both buffers
    for (int sp = 0; sp < c.n_species; ++sp) {
        std::vector<long long> start;
        std::vector<int> seg;
        const std::vector<long long> cnt = load_counts(&c, L.nxs, L.ntx, L.nty, sp);
        const std::vector<long long> extra = window_room(c, L, sp, 0);
        if (!layout_from_counts(cnt, L.pool[sp], L.maxseg[sp], &start, &seg, &extra))
            return fail(PIC_E_CAPACITY, "the initial load exceeds the particle slots");
        int rc = upload_layout(d.sp[sp], start, seg, std::vector<int>(cnt.begin(), cnt.end()), st);
        if (rc) return rc;
    }
    if (c.load)
        for (int sp = 0; sp < c.n_species; ++sp) HIPCHK(Launch<R>::load(d, sp, st));
    int rc = gauss_baseline(s, d, st);
    if (rc) return rc;
    rc = read_state(s, st);
    if (rc) return rc;
    if (s->hs.err & ERR_CAPACITY)
        return fail(PIC_E_CAPACITY, "initial load exceeds the tile capacity");
    return PIC_OK;
}

template <typename R>
int do_energy(pic_sim *s, const SimDev<R> &d, pic_diag *out, hipStream_t st)
{
    int rc = enqueue_settle(s, d, st);
    if (rc) return rc;
    rc = read_state(s, st);
    if (rc) return rc;
    const int has_prev = s->rho_prev_iter == s->hs.iter - 1;
    rc = enqueue_rho(d, st);
    if (rc) return rc;
    HIPCHK(Launch<R>::diag(d, has_prev, st));
    HIPCHK(Launch<R>::copy_plane(d.rho, d.rho_prev, (long long)d.nxs * d.ny, st));
    double res[N_RED];
    HIPCHK(hipMemcpyAsync(res, d.res, sizeof(res), hipMemcpyDeviceToHost, st));
    std::vector<int> cnt((size_t)s->L.ntiles);
    std::memset(out, 0, sizeof(*out));
    double charge = 0;
    for (int sp = 0; sp < d.nsp; ++sp) {
        HIPCHK(hipMemcpyAsync(cnt.data(), d.sp[sp].pb[s->hs.ppar].count, cnt.size() * 4,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        long long n = 0;
        for (int v : cnt) n += v;
        out->n_particles[sp] = n;
        const pic_species_cfg &p = s->cfg.sp[sp];
        const double qp = (p.q_over_m < 0 ? -1.0 : 1.0) * p.density / (p.ppc_x * p.ppc_y);
        charge += qp * (double)n * d.dx_d * d.dy_d;
    }
    HIPCHK(hipStreamSynchronize(st));
    s->rho_prev_iter = s->hs.iter;
    out->e_energy = res[0];
    out->b_energy = res[1];
    double ke = 0;
    for (int sp = 0; sp < d.nsp; ++sp) {
        out->ke[sp] = res[2 + sp];
        ke += res[2 + sp];
    }
    out->total = res[0] + res[1] + ke;
    out->charge = charge;
    out->gauss_res_max = res[6];
    out->cont_res_max = has_prev ? res[7] : -1.0;
    out->rho_max = res[8];
    out->step = s->hs.iter;
    out->t = (double)s->hs.iter * d.dt_d;
    out->nshift = s->hs.nshift;
    out->status = (s->hs.err & ERR_CAPACITY) ? PIC_E_CAPACITY : PIC_OK;
    return PIC_OK;
}

template <typename R>
int do_set_particles(pic_sim *s, const SimDev<R> &d, int sp, long long n, const int *ix,
                     const int *iy, const double *x, const double *y, const double *ux,
                     const double *uy, const double *uz, hipStream_t st)
{
    const pic_cfg &c = s->cfg;
    const Layout &L = s->L;
    int rc = enqueue_settle(s, d, st);
    if (rc) return rc;
    rc = read_state(s, st);
    if (rc) return rc;
    const int origin = s->hs.origin;
    std::vector<int> tile((size_t)n), cnt((size_t)L.ntiles, 0);
    for (long long k = 0; k < n; ++k) {
        if (ix[k] < 0 || ix[k] >= c.nx || iy[k] < 0 || iy[k] >= c.ny || !(x[k] >= 0.0) ||
            !(x[k] < 1.0) || !(y[k] >= 0.0) || !(y[k] < 1.0) || !std::isfinite(ux[k]) ||
            !std::isfinite(uy[k]) || !std::isfinite(uz[k]))
            return fail(PIC_E_ARG, "particle " + std::to_string(k) + " out of range");
        const int gx = c.moving_window ? (ix[k] + origin) % L.nxs : ix[k];
        tile[k] = gx / TX + (iy[k] / TY) * L.ntx;
        cnt[tile[k]] += 1;
    }
    // the tiles' segments from these counts, the same in both buffers
    std::vector<long long> sstart;
    std::vector<int> sseg;
    const std::vector<long long> extra = window_room(c, L, sp, origin);
    if (!layout_from_counts(std::vector<long long>(cnt.begin(), cnt.end()), L.pool[sp],
                            L.maxseg[sp], &sstart, &sseg, &extra))
        return fail(PIC_E_CAPACITY, "the particles exceed the species' particle slots (or a "
                                    "tile's largest segment)");
    rc = upload_layout(d.sp[sp], sstart, sseg, cnt, st);
    if (rc) return rc;
    // counting sort by tile, then one copy per array per non-empty tile
    std::vector<long long> start((size_t)L.ntiles + 1, 0);
    for (int t = 0; t < L.ntiles; ++t) start[t + 1] = start[t] + cnt[t];
    std::vector<long long> fillp(start.begin(), start.end() - 1);
    std::vector<int> hc((size_t)n);
    std::vector<R> hx((size_t)n), hy((size_t)n), hux((size_t)n), huy((size_t)n), huz((size_t)n);
    for (long long k = 0; k < n; ++k) {
        const long long q = fillp[tile[k]]++;
        const int gx = c.moving_window ? (ix[k] + origin) % L.nxs : ix[k];
        R xr = (R)x[k], yr = (R)y[k];
        if (xr >= R(1)) xr = std::nextafter(R(1), R(0));  // rounding must stay in [0, 1)
        if (yr >= R(1)) yr = std::nextafter(R(1), R(0));
        hc[q] = (int)((unsigned)gx | ((unsigned)iy[k] << 16));
        hx[q] = xr;
        hy[q] = yr;
        hux[q] = (R)ux[k];
        huy[q] = (R)uy[k];
        huz[q] = (R)uz[k];
    }
    const PartBuf<R> &P = d.sp[sp].pb[s->hs.ppar];
    for (int t = 0; t < L.ntiles; ++t) {
        if (!cnt[t]) continue;
        const size_t dst = (size_t)sstart[t], src = (size_t)start[t], m = (size_t)cnt[t];
        HIPCHK(hipMemcpyAsync(P.cell + dst, hc.data() + src, m * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(P.x + dst, hx.data() + src, m * sizeof(R), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(P.y + dst, hy.data() + src, m * sizeof(R), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(P.ux + dst, hux.data() + src, m * sizeof(R), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(P.uy + dst, huy.data() + src, m * sizeof(R), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(P.uz + dst, huz.data() + src, m * sizeof(R), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(P.count, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return gauss_baseline(s, d, st);
}

template <typename R>
int do_get_particles(pic_sim *s, const SimDev<R> &d, int sp, long long cap, long long *n_out,
                     int *ix, int *iy, double *x, double *y, double *ux, double *uy, double *uz,
                     hipStream_t st)
{
    const Layout &L = s->L;
    int rc = enqueue_settle(s, d, st);
    if (rc) return rc;
    rc = read_state(s, st);
    if (rc) return rc;
    const PartBuf<R> &P = d.sp[sp].pb[s->hs.ppar];
    std::vector<int> cnt((size_t)L.ntiles);
    std::vector<long long> sstart((size_t)L.ntiles);
    HIPCHK(hipMemcpyAsync(cnt.data(), P.count, cnt.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sstart.data(), d.sp[sp].start[s->hs.ppar], sstart.size() * 8,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    long long n = 0;
    for (int v : cnt) n += v;
    if (n_out) *n_out = n;
    if (!ix) return PIC_OK;
    if (n > cap) return fail(PIC_E_ARG, "output arrays too small");
    std::vector<int> hc((size_t)n);
    std::vector<R> hx((size_t)n), hy((size_t)n), hux((size_t)n), huy((size_t)n), huz((size_t)n);
    long long q = 0;
    for (int t = 0; t < L.ntiles; ++t) {
        if (!cnt[t]) continue;
        const size_t src = (size_t)sstart[t], m = (size_t)cnt[t];
        HIPCHK(hipMemcpyAsync(hc.data() + q, P.cell + src, m * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hx.data() + q, P.x + src, m * sizeof(R), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hy.data() + q, P.y + src, m * sizeof(R), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hux.data() + q, P.ux + src, m * sizeof(R), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(huy.data() + q, P.uy + src, m * sizeof(R), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(huz.data() + q, P.uz + src, m * sizeof(R), hipMemcpyDeviceToHost, st));
        q += (long long)m;
    }
    HIPCHK(hipStreamSynchronize(st));
    const int origin = s->hs.origin;
    for (long long k = 0; k < n; ++k) {
        const int gx = hc[k] & 0xffff;
        ix[k] = s->cfg.moving_window ? (gx - origin + L.nxs) % L.nxs : gx;
        iy[k] = (int)((unsigned)hc[k] >> 16);
        x[k] = hx[k];
        y[k] = hy[k];
        ux[k] = hux[k];
        uy[k] = huy[k];
        uz[k] = huz[k];
    }
    return PIC_OK;
}

// Host (ny, nx) window planes <-> device storage planes.
// lag = 1 maps with the window origin before the last step's shift (the
// current of a step lives in the window it was deposited in).
template <typename R>
int do_planes(pic_sim *s, R *const *dev, int np, double *host, bool to_dev, hipStream_t st,
              int lag = 0)
{
    const Layout &L = s->L;
    const pic_cfg &c = s->cfg;
    int rc = read_state(s, st);
    if (rc) return rc;
    const int origin = (s->hs.origin - (lag ? s->hs.shift : 0) + L.nxs) % L.nxs;
    std::vector<R> h(L.plane);
    const size_t hp = (size_t)c.nx * c.ny;
    for (int k = 0; k < np; ++k) {
        if (to_dev) {
            std::fill(h.begin(), h.end(), R(0));
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const int gx = c.moving_window ? (i + origin) % L.nxs : i;
                    h[(size_t)gx + (size_t)j * L.nxs] = (R)host[k * hp + (size_t)j * c.nx + i];
                }
            HIPCHK(hipMemcpyAsync(dev[k], h.data(), L.plane * sizeof(R), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        } else {
            HIPCHK(hipMemcpyAsync(h.data(), dev[k], L.plane * sizeof(R), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const int gx = c.moving_window ? (i + origin) % L.nxs : i;
                    host[k * hp + (size_t)j * c.nx + i] = (double)h[(size_t)gx + (size_t)j * L.nxs];
                }
        }
    }
    return PIC_OK;
}

// Steps replayed from captured graphs: one of GRAPH_STEPS steps (the first
// of them rewriting the push's work order) while that many remain, then
// one-step graphs (fewer graph launches, and no gap between the steps inside
// one graph).

template <typename R>
int capture_steps(pic_sim *s, const SimDev<R> &d, int k, hipGraph_t *graph, hipGraphExec_t *exec)
{
    if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
    int rc = PIC_OK;
    for (int n = 0; n < k && rc == PIC_OK; ++n)
        rc = enqueue_step(s, d, s->cap_stream, n == 0 && k == GRAPH_STEPS);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return fail(PIC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    *graph = g;
    HIPCHK(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return PIC_OK;
}

template <typename R>
int do_step(pic_sim *s, const SimDev<R> &d, int nsteps, hipStream_t st)
{
    if (s->timing) {
        for (int n = 0; n < nsteps; ++n) {
            const bool order = s->since_order >= GRAPH_STEPS;
            s->since_order = order ? 1 : s->since_order + 1;
            int rc = enqueue_step(s, d, st, order);
            if (rc) return rc;
        }
        return PIC_OK;
    }
    // both graphs on the first call, so that later calls only replay
    if (!s->gexec_n) {
        const int rc = capture_steps(s, d, GRAPH_STEPS, &s->graph_n, &s->gexec_n);
        if (rc) return rc;
    }
    if (!s->gexec) {
        const int rc = capture_steps(s, d, 1, &s->graph, &s->gexec);
        if (rc) return rc;
    }
    for (int n = 0; n < nsteps / GRAPH_STEPS; ++n) HIPCHK(hipGraphLaunch(s->gexec_n, st));
    if (nsteps >= GRAPH_STEPS) s->since_order = GRAPH_STEPS;  // the last graph's order
    for (int n = 0; n < nsteps % GRAPH_STEPS; ++n) {
        // one-step graphs hold no work order: launch one directly when due
        if (s->since_order >= GRAPH_STEPS) {
            HIPCHK(Launch<R>::order(d, st));
            s->since_order = 0;
        }
        HIPCHK(hipGraphLaunch(s->gexec, st));
        ++s->since_order;
    }
    return PIC_OK;
}

// The step filters the current inside the Yee launch, so a request for the
// filtered current filters the last step's J into Jf first (same arithmetic).
template <typename R>
int get_current(pic_sim *sim, const SimDev<R> &d, int filtered, double *j3, hipStream_t st)
{
    if (filtered && d.npass > 0) {
        const int rc = timed(sim, 3, st, [&] {
            return Launch<R>::filter(d, 3, d.J[0], d.J[1], d.J[2], d.Jf[0], d.Jf[1], d.Jf[2], st,
                                     true);
        });
        if (rc) return rc;
    }
    return do_planes(sim, filtered ? d.Jf : d.J, 3, j3, false, st, 1);
}

}  // namespace

#define DISPATCH(sim, call_f, call_d) ((sim)->cfg.fp64 ? (call_d) : (call_f))

extern "C" {

size_t pic_mem_bytes(const pic_cfg *cfg)
{
    return guarded<size_t>([&]() -> size_t {
        Layout L;
        if (layout(cfg, &L) != PIC_OK) return 0;
        return L.total;
    });
}

int pic_init(const pic_cfg *cfg, void *arena, size_t arena_bytes, void *stream, pic_sim **out)
{
    return guarded<int>([&]() -> int {
        if (!out) return fail(PIC_E_ARG, "out is NULL");
        *out = nullptr;
        Layout L;
        int rc = layout(cfg, &L);
        if (rc) return rc;
        if (!arena) return fail(PIC_E_ARG, "arena is NULL");
        if (((uintptr_t)arena) & 255) return fail(PIC_E_ARG, "arena must be 256-byte aligned");
        if (arena_bytes < L.total)
            return fail(PIC_E_NOMEM, "arena holds " + std::to_string(arena_bytes) + " bytes, needs " +
                                         std::to_string(L.total));
        // released to the caller on success; pic_free on any failure, thrown or returned
        std::unique_ptr<pic_sim, int (*)(pic_sim *)> own(new pic_sim(), pic_free);
        pic_sim *s = own.get();
        s->uid = g_next_uid.fetch_add(1);
        s->cfg = *cfg;
        s->L = L;
        s->arena = (char *)arena;
        std::memset(s->ms, 0, sizeof(s->ms));
        std::memset(s->launches, 0, sizeof(s->launches));
        hipStream_t st = (hipStream_t)stream;
        if (cfg->fp64) {
            describe(cfg, L, s->arena, &s->dd);
            rc = do_init(s, s->dd, st);
        } else {
            describe(cfg, L, s->arena, &s->df);
            rc = do_init(s, s->df, st);
        }
        if (rc) return rc;
        *out = own.release();
        return PIC_OK;
    });
}

int pic_deposit(pic_sim *sim, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim) return fail(PIC_E_ARG, "sim is NULL");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim, enqueue_deposit(sim, sim->df, st), enqueue_deposit(sim, sim->dd, st));
    });
}

int pic_field_advance(pic_sim *sim, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim) return fail(PIC_E_ARG, "sim is NULL");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim, enqueue_field_advance(sim, sim->df, st),
                        enqueue_field_advance(sim, sim->dd, st));
    });
}

int pic_step(pic_sim *sim, int nsteps, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || nsteps < 0) return fail(PIC_E_ARG, "bad sim or nsteps");
        if (nsteps == 0) return PIC_OK;
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim, do_step(sim, sim->df, nsteps, st), do_step(sim, sim->dd, nsteps, st));
    });
}

int pic_energy(pic_sim *sim, pic_diag *out, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || !out) return fail(PIC_E_ARG, "sim or out is NULL");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim, do_energy(sim, sim->df, out, st), do_energy(sim, sim->dd, out, st));
    });
}

int pic_status(pic_sim *sim, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim) return fail(PIC_E_ARG, "sim is NULL");
        int rc = read_state(sim, (hipStream_t)stream);
        if (rc) return rc;
        const int e = sim->hs.err;
        if (e & ERR_CAPACITY) {
            std::string what;
            const char *names[] = {"a tile's segment", "a tile's outbox", "a push block's arrival list",
                                   "a segment while settling leavers", "the pool for a relayout",
                                   "a segment while loading the window's new column",
                                   "a segment during the initial load"};
            for (int b = 0; b < 7; ++b)
                if (e & (1 << b)) what += (what.empty() ? "" : ", ") + std::string(names[b]);
            return fail(PIC_E_CAPACITY, "particle slots ran out: " + what);
        }
        return PIC_OK;
    });
}

int pic_free(pic_sim *sim)
{
    if (!sim) return PIC_OK;
    if (sim->gexec) (void)hipGraphExecDestroy(sim->gexec);
    if (sim->graph) (void)hipGraphDestroy(sim->graph);
    if (sim->gexec_n) (void)hipGraphExecDestroy(sim->gexec_n);
    if (sim->graph_n) (void)hipGraphDestroy(sim->graph_n);
    if (sim->cap_stream) (void)hipStreamDestroy(sim->cap_stream);
    for (hipEvent_t e : sim->ev) (void)hipEventDestroy(e);
    delete sim;
    return PIC_OK;
}

int pic_set_particles(pic_sim *sim, int sp, long long n, const int *ix, const int *iy,
                      const double *x, const double *y, const double *ux, const double *uy,
                      const double *uz, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || sp < 0 || sp >= sim->cfg.n_species || n < 0)
            return fail(PIC_E_ARG, "bad sim, species or count");
        if (n > 0 && (!ix || !iy || !x || !y || !ux || !uy || !uz))
            return fail(PIC_E_ARG, "NULL particle array");
        if (n > (long long)sim->L.pool[sp])
            return fail(PIC_E_CAPACITY, "more particles than the species has slots");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim,
                        do_set_particles(sim, sim->df, sp, n, ix, iy, x, y, ux, uy, uz, st),
                        do_set_particles(sim, sim->dd, sp, n, ix, iy, x, y, ux, uy, uz, st));
    });
}

long long pic_particle_count(pic_sim *sim, int sp, void *stream)
{
    return guarded<long long>([&]() -> long long {
        if (!sim || sp < 0 || sp >= sim->cfg.n_species) return fail(PIC_E_ARG, "bad sim or species");
        long long n = 0;
        hipStream_t st = (hipStream_t)stream;
        int rc = DISPATCH(sim,
                          do_get_particles(sim, sim->df, sp, 0, &n, nullptr, nullptr, nullptr,
                                           nullptr, nullptr, nullptr, nullptr, st),
                          do_get_particles(sim, sim->dd, sp, 0, &n, nullptr, nullptr, nullptr,
                                           nullptr, nullptr, nullptr, nullptr, st));
        return rc ? rc : n;
    });
}

int pic_get_particles(pic_sim *sim, int sp, long long cap, long long *n_out, int *ix, int *iy,
                      double *x, double *y, double *ux, double *uy, double *uz, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || sp < 0 || sp >= sim->cfg.n_species || !ix || !iy || !x || !y || !ux || !uy ||
            !uz)
            return fail(PIC_E_ARG, "bad sim, species or NULL array");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim,
                        do_get_particles(sim, sim->df, sp, cap, n_out, ix, iy, x, y, ux, uy, uz, st),
                        do_get_particles(sim, sim->dd, sp, cap, n_out, ix, iy, x, y, ux, uy, uz, st));
    });
}

int pic_set_fields(pic_sim *sim, const double *f6, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || !f6) return fail(PIC_E_ARG, "bad sim or NULL planes");
        hipStream_t st = (hipStream_t)stream;
        int rc = read_state(sim, st);
        if (rc) return rc;
        const int par = sim->hs.parity;
        if (sim->cfg.fp64) {
            rc = do_planes(sim, sim->dd.F[par], 6, (double *)f6, true, st);
            if (!rc) rc = gauss_baseline(sim, sim->dd, st);
        } else {
            rc = do_planes(sim, sim->df.F[par], 6, (double *)f6, true, st);
            if (!rc) rc = gauss_baseline(sim, sim->df, st);
        }
        return rc;
    });
}

int pic_get_fields(pic_sim *sim, double *f6, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || !f6) return fail(PIC_E_ARG, "bad sim or NULL planes");
        hipStream_t st = (hipStream_t)stream;
        int rc = read_state(sim, st);
        if (rc) return rc;
        const int par = sim->hs.parity;
        return DISPATCH(sim, do_planes(sim, sim->df.F[par], 6, f6, false, st),
                        do_planes(sim, sim->dd.F[par], 6, f6, false, st));
    });
}

int pic_get_current(pic_sim *sim, int filtered, double *j3, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || !j3) return fail(PIC_E_ARG, "bad sim or NULL planes");
        hipStream_t st = (hipStream_t)stream;
        return DISPATCH(sim, get_current(sim, sim->df, filtered, j3, st),
                        get_current(sim, sim->dd, filtered, j3, st));
    });
}

int pic_set_time(pic_sim *sim, long long iter, int nshift, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || iter < 0 || nshift < 0) return fail(PIC_E_ARG, "bad sim, iter or nshift");
        hipStream_t st = (hipStream_t)stream;
        int rc = read_state(sim, st);
        if (rc) return rc;
        sim->hs.iter = iter;
        sim->hs.nshift = nshift;
        sim->rho_prev_iter = -2;
        return write_state(sim, st);
    });
}

int pic_timing(pic_sim *sim, int enable, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim) return fail(PIC_E_ARG, "sim is NULL");
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        sim->timing = enable != 0;
        sim->ev_used = 0;
        if (enable) {
            std::memset(sim->ms, 0, sizeof(sim->ms));
            std::memset(sim->launches, 0, sizeof(sim->launches));
        }
        return PIC_OK;
    });
}

int pic_timing_read(pic_sim *sim, double *ms, long long *launches, int nk, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!sim || nk < 0) return fail(PIC_E_ARG, "bad sim or nk");
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        int rc = timing_flush(sim);
        if (rc) return rc;
        for (int k = 0; k < nk && k < PIC_NK; ++k) {
            if (ms) ms[k] = sim->ms[k];
            if (launches) launches[k] = sim->launches[k];
        }
        return PIC_OK;
    });
}

int pic_layout(const pic_sim *sim, long long *out, int n)
{
    return guarded<int>([&]() -> int {
        if (!sim || !out) return fail(PIC_E_ARG, "bad sim or out");
        const long long v[7] = {TX, TY, sim->L.ntx, sim->L.nty, sim->L.nxs,
                                sim->cfg.n_species ? (long long)sim->L.pool[0] : 0LL,
                                (long long)sim->L.cap_out};
        for (int k = 0; k < n && k < 7; ++k) out[k] = v[k];
        return PIC_OK;
    });
}

const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_E_ARG: return "invalid argument";
    case PIC_E_CFL: return "timestep violates the Courant limit";
    case PIC_E_NOMEM: return "arena too small";
    case PIC_E_CAPACITY: return "particle capacity exceeded";
    case PIC_E_HIP: return "HIP runtime error";
    case PIC_E_STATE: return "invalid state";
    case PIC_E_CANCELLED: return "cancelled";
    default: return "unknown error";
    }
}

const char *pic_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ===========================================================================
// batches of simulations
// ===========================================================================
struct pic_batch {
    char *arena = nullptr;
    int max_sims = 0;
    long long max_tiles = 0;
    SimDev<float> *d_table = nullptr;
    BatchDev *d_batch = nullptr;
    int2 *d_work = nullptr;
    int2 *d_fwork = nullptr;  // units of the streaming fold
    int2 *d_ywork = nullptr;  // units of the streaming filter + Yee
    SimDev<float> *h_table = nullptr;  // pinned staging
    BatchDev *h_batch = nullptr;
    int2 *h_work = nullptr;
    int2 *h_fwork = nullptr;
    int2 *h_ywork = nullptr;
    std::vector<unsigned long long> cur;  // uids of the staged simulations
    int grid = 0, grid_fold = 0, grid_yee = 0;
    int rf = -2;  // filter halo of the captured graph (-1: tile forms)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace {

// Units of the streaming field kernels per simulation: the fold's are at
// most 2 ntx nty + 2 nty <= 4 ntiles, the filter + Yee's at most ntx * 3 nty
// (strips of >= 55 columns and 6 rows), so lists of 4 max_tiles hold both.
constexpr int SUNITS_PER_TILE = 4;

void batch_layout(int max_sims, long long max_tiles, size_t *o_table, size_t *o_batch,
                  size_t *o_work, size_t *o_fwork, size_t *o_ywork, size_t *total)
{
    size_t o = 0;
    *o_table = o;
    o = align256(o + (size_t)max_sims * sizeof(SimDev<float>));
    *o_batch = o;
    o = align256(o + sizeof(BatchDev));
    *o_work = o;
    o = align256(o + (size_t)max_tiles * sizeof(int2));
    *o_fwork = o;
    o = align256(o + (size_t)max_tiles * SUNITS_PER_TILE * sizeof(int2));
    *o_ywork = o;
    o = align256(o + (size_t)max_tiles * SUNITS_PER_TILE * sizeof(int2));
    *total = o;
}

// Before each batched step: the particle layouts of every member (one
// launch over the descriptor table) once any member has taken GRAPH_STEPS
// pushes since its last check, the cadence of pic_step; then every member
// counts the step.
hipError_t batch_layouts(pic_sim *const *sims, int n, const SimDev<float> *table, hipStream_t st)
{
    bool due = false;
    for (int i = 0; i < n; ++i) due |= sims[i]->since_order >= GRAPH_STEPS;
    if (due) {
        const hipError_t e = Launch<float>::layout_b(table, n, st);
        if (e != hipSuccess) return e;
        for (int i = 0; i < n; ++i) sims[i]->since_order = 0;
    }
    for (int i = 0; i < n; ++i) ++sims[i]->since_order;
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t pic_batch_mem_bytes(int max_sims, long long max_tiles)
{
    return guarded<size_t>([&]() -> size_t {
        if (max_sims < 1 || max_tiles < 1) return 0;
        size_t a, b, c, f, y, t;
        batch_layout(max_sims, max_tiles, &a, &b, &c, &f, &y, &t);
        return t;
    });
}

int pic_batch_free(pic_batch *b)
{
    if (!b) return PIC_OK;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_table) (void)hipHostFree(b->h_table);
    if (b->h_batch) (void)hipHostFree(b->h_batch);
    if (b->h_work) (void)hipHostFree(b->h_work);
    if (b->h_fwork) (void)hipHostFree(b->h_fwork);
    if (b->h_ywork) (void)hipHostFree(b->h_ywork);
    delete b;
    return PIC_OK;
}

int pic_batch_create(void *arena, size_t arena_bytes, int max_sims, long long max_tiles,
                     pic_batch **out)
{
    return guarded<int>([&]() -> int {
        if (!out) return fail(PIC_E_ARG, "out is NULL");
        *out = nullptr;
        if (!arena || ((uintptr_t)arena & 255) || max_sims < 1 || max_tiles < 1)
            return fail(PIC_E_ARG, "bad batch arena or sizes");
        size_t ot, ob, ow, of, oy, total;
        batch_layout(max_sims, max_tiles, &ot, &ob, &ow, &of, &oy, &total);
        if (arena_bytes < total) return fail(PIC_E_NOMEM, "batch arena too small");
        pic_batch *b = new pic_batch();
        b->arena = (char *)arena;
        b->max_sims = max_sims;
        b->max_tiles = max_tiles;
        b->d_table = (SimDev<float> *)(b->arena + ot);
        b->d_batch = (BatchDev *)(b->arena + ob);
        b->d_work = (int2 *)(b->arena + ow);
        b->d_fwork = (int2 *)(b->arena + of);
        b->d_ywork = (int2 *)(b->arena + oy);
        hipError_t e = hipHostMalloc((void **)&b->h_table, (size_t)max_sims * sizeof(SimDev<float>));
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_batch, sizeof(BatchDev));
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_work, (size_t)max_tiles * sizeof(int2));
        const size_t su = (size_t)max_tiles * SUNITS_PER_TILE * sizeof(int2);
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_fwork, su);
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_ywork, su);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            pic_batch_free(b);
            return fail(PIC_E_HIP, std::string("batch set-up: ") + hipGetErrorString(e));
        }
        *out = b;
        return PIC_OK;
    });
}

int pic_batch_step(pic_batch *b, pic_sim *const *sims, int n, int nsteps, void *stream)
{
    return guarded<int>([&]() -> int {
        if (!b || n < 0 || nsteps < 0 || (n > 0 && !sims)) return fail(PIC_E_ARG, "bad batch call");
        if (n == 0 || nsteps == 0) return PIC_OK;
        if (n > b->max_sims) return fail(PIC_E_ARG, "more simulations than the batch holds");
        hipStream_t st = (hipStream_t)stream;
        bool same = (int)b->cur.size() == n;
        for (int i = 0; same && i < n; ++i) same = sims[i] && sims[i]->uid == b->cur[i];
        if (!same) {
            long long nwork = 0;
            for (int i = 0; i < n; ++i) {
                const pic_sim *s = sims[i];
                if (!s || s->cfg.fp64 || s->cfg.moving_window || s->cfg.deposit_mode != 0)
                    return fail(PIC_E_ARG, "batches hold FP32 periodic simulations with the "
                                           "reduction deposit only");
                nwork += s->L.ntiles;
            }
            if (nwork > b->max_tiles) return fail(PIC_E_ARG, "batch work list too long");
            // the streaming field kernels need one filter halo for the whole batch
            int rf = -1;
            for (int i = 0; i < n; ++i) {
                const pic_cfg &c = sims[i]->cfg;
                const int r = c.filter_passes > 0 ? c.filter_passes + (c.filter_compensate ? 1 : 0) : 0;
                rf = i == 0 ? r : (r == rf ? rf : -1);
                if (rf < 0) break;
            }
            // the staging buffers may still feed an earlier copy
            HIPCHK(hipStreamSynchronize(st));
            long long w = 0, wf = 0, wy = 0;
            for (int i = 0; i < n; ++i) {
                const Layout &L = sims[i]->L;
                b->h_table[i] = sims[i]->df;
                b->h_table[i].nsb = 1;  // batched pushes take every species of a tile at once
                for (int t = 0; t < L.ntiles; ++t) b->h_work[w++] = make_int2(i, t);
                if (rf >= 0) {
                    const int nf = fold_units(L.ntx, L.nty), ny = yee_units(L.nxs, sims[i]->cfg.ny, rf);
                    if (wf + nf > b->max_tiles * SUNITS_PER_TILE || wy + ny > b->max_tiles * SUNITS_PER_TILE)
                        return fail(PIC_E_ARG, "batch work list too long");
                    for (int u = 0; u < nf; ++u) b->h_fwork[wf++] = make_int2(i, u);
                    for (int u = 0; u < ny; ++u) b->h_ywork[wy++] = make_int2(i, u);
                }
            }
            b->h_batch->nwork = (int)nwork;
            b->h_batch->nsim = n;
            b->h_batch->work = b->d_work;
            b->h_batch->blocks_done = 0;
            b->h_batch->nfold = (int)wf;
            b->h_batch->nyee = (int)wy;
            b->h_batch->fold_work = b->d_fwork;
            b->h_batch->yee_work = b->d_ywork;
            HIPCHK(hipMemcpyAsync(b->d_table, b->h_table, (size_t)n * sizeof(SimDev<float>),
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(b->d_work, b->h_work, (size_t)nwork * sizeof(int2),
                                  hipMemcpyHostToDevice, st));
            if (rf >= 0) {
                HIPCHK(hipMemcpyAsync(b->d_fwork, b->h_fwork, (size_t)wf * sizeof(int2),
                                      hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(b->d_ywork, b->h_ywork, (size_t)wy * sizeof(int2),
                                      hipMemcpyHostToDevice, st));
            }
            HIPCHK(hipMemcpyAsync(b->d_batch, b->h_batch, sizeof(BatchDev), hipMemcpyHostToDevice,
                                  st));
            b->cur.resize(n);
            for (int i = 0; i < n; ++i) b->cur[i] = sims[i]->uid;
            // one graph serves every work list up to its grid; blocks past the
            // work count exit at once
            auto round = [](long long v) { return (int)((v + 1023) / 1024 * 1024); };
            const int need = round(nwork), need_f = round(wf), need_y = round(wy);
            auto fits = [](int need_, int grid_) { return need_ <= grid_ && grid_ <= 4 * need_; };
            if (!b->gexec || rf != b->rf || !fits(need, b->grid) ||
                (rf >= 0 && (!fits(need_f, b->grid_fold) || !fits(need_y, b->grid_yee)))) {
                if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
                if (b->graph) (void)hipGraphDestroy(b->graph);
                b->gexec = nullptr;
                b->graph = nullptr;
                HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
                hipError_t le = launch_batch_step<float>(b->d_table, b->d_batch, need, b->cap_stream,
                                                         rf, need_f, need_y);
                hipGraph_t g = nullptr;
                hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
                if (le != hipSuccess || ce != hipSuccess)
                    return fail(PIC_E_HIP, "batch graph capture failed");
                b->graph = g;
                HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
                b->grid = need;
                b->grid_fold = need_f;
                b->grid_yee = need_y;
                b->rf = rf;
            }
        }
        for (int k = 0; k < nsteps; ++k) {
            HIPCHK(batch_layouts(sims, n, b->d_table, st));
            HIPCHK(hipGraphLaunch(b->gexec, st));
        }
        return PIC_OK;
    });
}

}  // extern "C"

// ===========================================================================
// batched steps that allocate nothing: the descriptor table, the batch
// descriptor and the work lists live in a file-scope device array instead of
// a batch object's arena
// ===========================================================================
namespace {

constexpr size_t align256c(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t ST_TABLE = 0;
constexpr size_t ST_BATCH = align256c(ST_TABLE + (size_t)PIC_STATIC_MAX_SIMS * sizeof(SimDev<float>));
constexpr size_t ST_WORK = align256c(ST_BATCH + sizeof(BatchDev));
constexpr size_t ST_FWORK = align256c(ST_WORK + (size_t)PIC_STATIC_MAX_TILES * sizeof(int2));
constexpr size_t ST_YWORK =
    align256c(ST_FWORK + (size_t)PIC_STATIC_MAX_TILES * SUNITS_PER_TILE * sizeof(int2));
constexpr size_t ST_BYTES =
    align256c(ST_YWORK + (size_t)PIC_STATIC_MAX_TILES * SUNITS_PER_TILE * sizeof(int2));

}  // namespace

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[ST_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES];  // device address of `scratch`, per device

// Device address of the current device's `scratch`, looked up once per device.
int scratch_address(void **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PIC_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PIC_OK;
}

// A descriptor written to device memory from a kernel argument.
template <typename T>
__global__ void k_put(T *dst, T src)
{
    static_assert(sizeof(T) % 4 == 0, "copied as 32-bit words");
    const unsigned *a = reinterpret_cast<const unsigned *>(&src);
    unsigned *b = reinterpret_cast<unsigned *>(dst);
    for (int k = threadIdx.x; k < (int)(sizeof(T) / 4); k += blockDim.x) b[k] = a[k];
}

// The three (simulation, unit) work lists from per-simulation counts:
// pre[l][i] is the first entry of simulation i in list l (l = 0: tiles of
// the push, 1: units of the streaming fold, 2: of the filter + Yee).
struct StaticLists {
    int n;
    int pre[3][PIC_STATIC_MAX_SIMS + 1];
};

__global__ __launch_bounds__(256) void k_lists(int2 *w0, int2 *w1, int2 *w2, StaticLists L)
{
    for (int l = 0; l < 3; ++l) {
        int2 *w = l == 0 ? w0 : (l == 1 ? w1 : w2);
        const int total = L.pre[l][L.n];
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total;
             k += gridDim.x * blockDim.x) {
            int i = 0;
            while (L.pre[l][i + 1] <= k) ++i;
            w[k] = make_int2(i, k - L.pre[l][i]);
        }
    }
}

}  // namespace

extern "C" {

int pic_batch_step_static(pic_sim *const *sims, int n, int nsteps, void *stream)
{
    return guarded<int>([&]() -> int {
        if (n < 0 || nsteps < 0 || (n > 0 && !sims)) return fail(PIC_E_ARG, "bad batch call");
        if (n == 0 || nsteps == 0) return PIC_OK;
        if (n > PIC_STATIC_MAX_SIMS)
            return fail(PIC_E_ARG, "pic_batch_step_static holds at most PIC_STATIC_MAX_SIMS (" +
                                       std::to_string(PIC_STATIC_MAX_SIMS) + ") simulations");
        StaticLists lists{};
        lists.n = n;
        int rf = -1;
        for (int i = 0; i < n; ++i) {
            const pic_sim *s = sims[i];
            if (!s || s->cfg.fp64 || s->cfg.moving_window || s->cfg.deposit_mode != 0)
                return fail(PIC_E_ARG, "batches hold FP32 periodic simulations with the "
                                       "reduction deposit only");
            const pic_cfg &c = s->cfg;
            const int r = c.filter_passes > 0 ? c.filter_passes + (c.filter_compensate ? 1 : 0) : 0;
            rf = i == 0 ? r : (r == rf ? rf : -1);
        }
        long long tot[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i) {
            const Layout &L = sims[i]->L;
            const long long cnt[3] = {L.ntiles, rf >= 0 ? fold_units(L.ntx, L.nty) : 0,
                                      rf >= 0 ? yee_units(L.nxs, sims[i]->cfg.ny, rf) : 0};
            for (int l = 0; l < 3; ++l) {
                lists.pre[l][i] = (int)tot[l];
                tot[l] += cnt[l];
            }
        }
        if (tot[0] > PIC_STATIC_MAX_TILES || tot[1] > PIC_STATIC_MAX_TILES * SUNITS_PER_TILE ||
            tot[2] > PIC_STATIC_MAX_TILES * SUNITS_PER_TILE)
            return fail(PIC_E_ARG, "pic_batch_step_static holds at most PIC_STATIC_MAX_TILES (" +
                                       std::to_string(PIC_STATIC_MAX_TILES) +
                                       ") tiles over all simulations");
        for (int l = 0; l < 3; ++l) lists.pre[l][n] = (int)tot[l];
        void *base = nullptr;
        int rc = scratch_address(&base);
        if (rc) return rc;
        char *sc = static_cast<char *>(base);
        SimDev<float> *table = reinterpret_cast<SimDev<float> *>(sc + ST_TABLE);
        BatchDev *bd = reinterpret_cast<BatchDev *>(sc + ST_BATCH);
        int2 *work = reinterpret_cast<int2 *>(sc + ST_WORK);
        int2 *fwork = reinterpret_cast<int2 *>(sc + ST_FWORK);
        int2 *ywork = reinterpret_cast<int2 *>(sc + ST_YWORK);
        hipStream_t st = (hipStream_t)stream;
        // stage everything on the stream: descriptors from kernel arguments,
        // work lists from the counts; the batch descriptor's completion count
        // starts at zero
        for (int i = 0; i < n; ++i) {
            SimDev<float> dsc = sims[i]->df;
            dsc.nsb = 1;  // batched pushes take every species of a tile at once
            hipLaunchKernelGGL(k_put<SimDev<float>>, dim3(1), dim3(256), 0, st, table + i, dsc);
            HIPCHK(hipGetLastError());
        }
        BatchDev b{};
        b.nwork = (int)tot[0];
        b.nsim = n;
        b.work = work;
        b.blocks_done = 0;
        b.nfold = (int)tot[1];
        b.nyee = (int)tot[2];
        b.fold_work = fwork;
        b.yee_work = ywork;
        hipLaunchKernelGGL(k_put<BatchDev>, dim3(1), dim3(64), 0, st, bd, b);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_lists, dim3(64), dim3(256), 0, st, work, fwork, ywork, lists);
        HIPCHK(hipGetLastError());
        for (int k = 0; k < nsteps; ++k) {
            HIPCHK(batch_layouts(sims, n, table, st));
            HIPCHK(launch_batch_step<float>(table, bd, (int)tot[0], st, rf, (int)tot[1],
                                            (int)tot[2]));
        }
        return PIC_OK;
    });
}

}  // extern "C"

// ===========================================================================
// serving loop
// ===========================================================================
namespace {

// First-fit allocator of 256-byte aligned ranges of the serving arena.
class ArenaAlloc {
  public:
    explicit ArenaAlloc(size_t bytes) { free_[0] = bytes & ~(size_t)255; }
    long long take(size_t bytes)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, left = it->second - bytes;
                free_.erase(it);
                if (left) free_[off + bytes] = left;
                return (long long)off;
            }
        }
        return -1;
    }
    void give(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

// Particles a configuration loads at initialisation (0 if it is invalid).
long long initial_particles(const pic_cfg *c)
{
    Layout L;
    if (layout(c, &L) != PIC_OK || !c->load) return 0;
    long long n = 0;
    for (int s = 0; s < c->n_species; ++s)
        if (c->sp[s].density > 0.0)
            for (long long v : load_counts(c, L.nxs, L.ntx, L.nty, s)) n += v;
    return n;
}

struct Active {
    int req;
    pic_sim *sim;
    size_t off, bytes;
    int left;
    double cost;  // relative work of one step (its arena size)
};

}  // namespace

extern "C" int pic_serve(const pic_request *reqs, int n, void *arena, size_t arena_bytes,
                         const pic_serve_opts *opts, pic_result *out, double *step_ms,
                         long long cap_steps, long long *n_steps, void *stream)
{
    return guarded<int>([&]() -> int {
        if (n < 0 || (n > 0 && (!reqs || !out)) || !arena || !opts || ((uintptr_t)arena & 255))
            return fail(PIC_E_ARG, "bad serving arguments");
        const int chunk = std::max(1, opts->chunk_steps);
        const int max_active = opts->batched ? (opts->max_batch > 0 ? opts->max_batch : 256) : 1;
        if (n_steps) *n_steps = 0;
        for (int i = 0; i < n; ++i) {
            std::memset(&out[i], 0, sizeof(out[i]));
            out[i].status = PIC_E_STATE;
        }
        // batch workspace at the start of the arena, the rest is the budget
        long long max_tiles = 0;
        for (int i = 0; i < n; ++i) {
            Layout L;
            if (layout(&reqs[i].cfg, &L) == PIC_OK) max_tiles += L.ntiles;
        }
        max_tiles = std::max(1LL, std::min(max_tiles, 1LL << 22));
        const size_t bws = align256(pic_batch_mem_bytes(max_active, max_tiles));
        if (arena_bytes < bws + 256) return fail(PIC_E_NOMEM, "budget smaller than the batch workspace");
        pic_batch *batch = nullptr;
        int rc = pic_batch_create(arena, bws, max_active, max_tiles, &batch);
        if (rc) return rc;
        hipStream_t sa = (hipStream_t)stream, sb = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t he = hipStreamCreateWithFlags(&sb, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreate(&e0);
        if (he == hipSuccess) he = hipEventCreate(&e1);
        auto teardown = [&] {
            (void)hipStreamSynchronize(sa);
            if (sb) (void)hipStreamSynchronize(sb);
            pic_batch_free(batch);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (sb) (void)hipStreamDestroy(sb);
        };
        if (he != hipSuccess) {
            teardown();
            return fail(PIC_E_HIP, std::string("serving set-up: ") + hipGetErrorString(he));
        }
        char *pool = (char *)arena + bws;
        const size_t pool_bytes = (arena_bytes - bws) & ~(size_t)255;
        ArenaAlloc alloc(pool_bytes);
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
        const auto t0 = std::chrono::steady_clock::now();
        auto now = [&] {
            return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        };
        // initial particle loads, for the running set's limit
        std::vector<long long> load(n, 0);
        if (opts->batched && opts->max_particles > 0)
            for (int i = 0; i < n; ++i) load[i] = initial_particles(&reqs[i].cfg);
        std::vector<int> queue;
        std::vector<Active> active;
        std::vector<pic_sim *> sims;
        int next = 0, done = 0;
        long long ns = 0;
        // admit queued requests, first fit in arrival order (one at a time: strictly
        // in order), initialising them on stream sb while the step stream runs
        auto admit = [&] {
            const double tnow = now();
            while (next < n && reqs[order[next]].arrival_s <= tnow) queue.push_back(order[next++]);
            for (size_t qi = 0; qi < queue.size() && (int)active.size() < max_active;) {
                const int r = queue[qi];
                const size_t need = pic_mem_bytes(&reqs[r].cfg);
                const bool unbatchable = opts->batched && (reqs[r].cfg.fp64 ||
                                                           reqs[r].cfg.moving_window ||
                                                           reqs[r].cfg.deposit_mode != 0);
                if (need == 0 || unbatchable || align256(need) > pool_bytes) {
                    out[r].status = need == 0 || unbatchable ? PIC_E_ARG : PIC_E_NOMEM;
                    ++done;
                    queue.erase(queue.begin() + qi);
                    continue;
                }
                if (opts->batched && opts->max_particles > 0 && !active.empty()) {
                    long long running = load[r];
                    for (const Active &a : active) running += load[a.req];
                    // no backlog behind this request: the lone limit
                    const bool lone = qi + 1 == queue.size();
                    const long long cap = lone && opts->lone_particles > 0
                                              ? opts->lone_particles
                                              : opts->max_particles;
                    if (running > cap) break;  // in arrival order
                }
                const long long off = alloc.take(need);
                if (off < 0) {
                    if (!opts->batched) break;
                    ++qi;
                    continue;
                }
                pic_sim *sim = nullptr;
                const int ir = pic_init(&reqs[r].cfg, pool + off, need, sb, &sim);
                queue.erase(queue.begin() + qi);
                if (ir) {
                    alloc.give((size_t)off, need);
                    out[r].status = ir;
                    ++done;
                    continue;
                }
                out[r].admit_s = now();
                active.push_back(Active{r, sim, (size_t)off, need, std::max(0, reqs[r].nsteps),
                                        (double)need});
            }
        };
        auto cancelled = [&](int r, double tnow) {
            return (reqs[r].cancel_s > 0 && tnow >= reqs[r].cancel_s) ||
                   (opts->cancel && opts->cancel[r] != 0);
        };
        // cancellation: queued requests are dropped, running ones retired with
        // the diagnostics of the steps they did (the step stream is idle here:
        // every chunk is waited for before the loop comes round)
        auto cancel = [&] {
            const double tnow = now();
            for (size_t qi = 0; qi < queue.size();) {
                const int r = queue[qi];
                if (!cancelled(r, tnow)) {
                    ++qi;
                    continue;
                }
                out[r].status = PIC_E_CANCELLED;
                out[r].done_s = tnow;
                ++done;
                queue.erase(queue.begin() + qi);
            }
            for (size_t ai = 0; ai < active.size();) {
                Active &a = active[ai];
                if (a.left <= 0 || !cancelled(a.req, tnow)) {
                    ++ai;
                    continue;
                }
                (void)pic_energy(a.sim, &out[a.req].diag, sa);
                out[a.req].status = PIC_E_CANCELLED;
                out[a.req].done_s = now();
                pic_free(a.sim);
                alloc.give(a.off, a.bytes);
                ++done;
                active.erase(active.begin() + ai);
            }
        };
        auto retire = [&] {
            for (size_t ai = 0; ai < active.size();) {
                Active &a = active[ai];
                if (a.left > 0) {
                    ++ai;
                    continue;
                }
                out[a.req].status = pic_energy(a.sim, &out[a.req].diag, sa);
                out[a.req].done_s = now();
                pic_free(a.sim);
                alloc.give(a.off, a.bytes);
                ++done;
                active.erase(active.begin() + ai);
            }
        };
        while (done < n && rc == PIC_OK) {
            admit();
            cancel();
            retire();
            if (active.empty()) {
                if (queue.empty() && next < n) {
                    const double wait = reqs[order[next]].arrival_s - now();
                    if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
                }
                continue;
            }
            // one chunk of the running set, all members in lockstep
            int k = chunk;
            sims.clear();
            for (const Active &a : active) {
                sims.push_back(a.sim);
                k = std::min(k, a.left);
            }
            (void)hipEventRecord(e0, sa);
            // a batch of one runs the simulation's own step graph
            rc = sims.size() > 1 ? pic_batch_step(batch, sims.data(), (int)sims.size(), k, sa)
                                 : pic_step(sims[0], k, sa);
            if (rc) break;
            // multi-rate: a request costing c times less than the largest one
            // takes min(c, rate_ratio) chunks' worth of steps, the extra ones
            // in shared launches of the cheaper requests only, k steps each
            std::vector<int> extra(active.size(), 0);
            if (opts->batched && opts->rate_ratio > 1 && active.size() > 1) {
                double cmax = 0;
                for (const Active &a : active) cmax = std::max(cmax, a.cost);
                int rounds = 0;
                for (size_t ai = 0; ai < active.size(); ++ai) {
                    const Active &a = active[ai];
                    const int rate = (int)std::min<double>(opts->rate_ratio, cmax / a.cost);
                    extra[ai] = std::max(0, std::min(rate - 1, (a.left - k) / k));
                    rounds = std::max(rounds, extra[ai]);
                }
                std::vector<pic_sim *> sub;
                for (int u = 1; u <= rounds && rc == PIC_OK; ++u) {
                    sub.clear();
                    long long tiles = 0;
                    for (size_t ai = 0; ai < active.size(); ++ai)
                        if (extra[ai] >= u && (int)sub.size() < PIC_STATIC_MAX_SIMS &&
                            tiles + active[ai].sim->L.ntiles <= PIC_STATIC_MAX_TILES) {
                            sub.push_back(active[ai].sim);
                            tiles += active[ai].sim->L.ntiles;
                        } else if (extra[ai] >= u) {
                            extra[ai] = u - 1;  // no room this round: fewer extra steps
                        }
                    if (!sub.empty())
                        rc = pic_batch_step_static(sub.data(), (int)sub.size(), k, sa);
                }
                if (rc) break;
            }
            (void)hipEventRecord(e1, sa);
            admit();  // while the chunk runs
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (step_ms && ns < cap_steps) step_ms[ns] = ms / k;
            ++ns;
            for (size_t ai = 0; ai < active.size(); ++ai) {
                Active &a = active[ai];
                if (std::find(sims.begin(), sims.end(), a.sim) != sims.end())
                    a.left -= k * (1 + (ai < extra.size() ? extra[ai] : 0));
            }
        }
        for (Active &a : active) pic_free(a.sim);
        if (n_steps) *n_steps = ns;
        teardown();
        return rc;
    });
}
