// C ABI: problem plan, workspace carving, step sequence, state I/O.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>
#include "adg_kernels.h"

using namespace adg;

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Worker threads of the host-side set-up loops (projection of initial data, initial
// detection): OMP_NUM_THREADS if set, else the hardware's, at most 16.
static int host_threads() {
    const char *e = std::getenv("OMP_NUM_THREADS");
    int n = e ? std::atoi(e) : 0;
    if (n <= 0) n = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 16));
}

// fn(lo, hi) on contiguous chunks of [0, n), one per worker thread.
template <class F>
static void parallel_for(int64_t n, F &&fn) {
    const int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(n / 64, 1));
    if (nt <= 1) {
        fn((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; t++) {
        const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([&fn, lo, hi] { fn(lo, hi); });
    }
    for (auto &x : th) x.join();
}

#define HIPCHK(call)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return fail(ADG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

struct adg_problem {
    Prob P;
    adg_params prm;
    Tables tab_host;
    int64_t cap;            // pool slots
    int chunk;              // workgroups (scratch slots) of the persistent subcell kernel
    int npos;               // subcell positions per troubled cell
    int lam_blocks;
    size_t ws_bytes;
    // offsets into the workspace
    struct Off {
        size_t tab, u0, u1, emin0, emax0, emin1, emax1, trace, gbar, beta0, beta1, force, mflag, margin, tlist, clist,
            slot0,
            slot1, pool0, pool1, sflux, blk, counts, scal, lampart, ring, halo, Y, strace, fpts, mask, big, end;
    } off;
    int64_t ring_cap = 0;    // ghost-ring cells of the extended grid (+ every cell, for solid cells)
    int64_t nring = 0;       // extended cells whose bounds the step computes (ghost ring on
                             // non-periodic sides, solid cells of the masked geometry)
    std::vector<uint8_t> mask;   // masked geometry, 1 = solid (empty: no solid cells)
    bool bounds_valid = false;  // interior old-time bounds were written by the previous step
    // bound state
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    Bufs B;
    Tables *tab_dev = nullptr;
    int cur = 0;
    bool bound = false, has_state = false;
    int *pinned = nullptr;    // host-pinned copy of the counters
    hipEvent_t counts_ready = nullptr;   // recorded after the asynchronous counter copy
    bool capturing = false;              // inside a batch graph capture
    struct adg_batch *batch = nullptr;   // the batch that steps this problem (set_state / step refused)
    bool batch_driving = false;          // the batch itself is calling the step functions
    int64_t nonphys_reported = 0;        // cumulative non-physical subcell results already reported
    int64_t last_troubled = 0, last_corrected = 0, steps = 0;
    // kernel-group timing
    unsigned prof_mask = 0;   // kernel groups timed (bit g: group g)
    struct Mark { int group; hipEvent_t a, b; };
    std::vector<Mark> pending;
    std::vector<hipEvent_t> spare;
    double prof_ms[8] = {0};
    int64_t prof_n[8] = {0};
};

static hipEvent_t take_event(adg_problem *pb) {
    if (!pb->spare.empty()) {
        hipEvent_t e = pb->spare.back();
        pb->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records events around one kernel group when that group is timed.
struct GroupTimer {
    adg_problem *pb;
    int group;
    hipEvent_t a = nullptr, b = nullptr;
    GroupTimer(adg_problem *p, int g) : pb(p), group(g) {
        if (!((pb->prof_mask >> g) & 1u)) return;
        a = take_event(pb);
        b = take_event(pb);
        if (a) (void)hipEventRecord(a, pb->stream);
    }
    ~GroupTimer() {
        if (!a || !b) return;
        (void)hipEventRecord(b, pb->stream);
        pb->pending.push_back({group, a, b});
    }
};

// Accumulates completed marks (the stream must have been synchronised).
static void harvest(adg_problem *pb) {
    for (auto &m : pb->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            pb->prof_ms[m.group] += ms;
            pb->prof_n[m.group] += 1;
        }
        pb->spare.push_back(m.a);
        pb->spare.push_back(m.b);
    }
    pb->pending.clear();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void plan(adg_problem *pb) {
    const Prob &P = pb->P;
    const int d = P.dim, nv = P.nv, n = P.n, Ns = P.Ns;
    const int64_t nn = ipow64(n, d), nfn = ipow64(n, d - 1), nsub = ipow64(Ns, d);
    int64_t next = 1;
    for (int j = 0; j < d; j++) next *= P.nc[j] + 2;
    const int64_t nc = P.ncell;
    const int64_t nblk = (nc + 255) / 256;
    const int64_t hsz = ipow64(Ns + 6, d), n3 = ipow64(3, d), nf3 = ipow64(3, d - 1);
    const int64_t per_chunk_cell = (nv * hsz + pb->npos * nv * n3 + pb->npos * 2 * d * nv * nf3 * 3) * 8;
    // subcell scratch: one slot per workgroup of the persistent subcell kernel (as many as
    // the 256 CUs of MI355X hold at once, fewer if the pool holds fewer cells)
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(subcell_workgroups(d, P.N, pb->prm.precision), pb->cap));
    if (big_slot_doubles(d, P.N) > 0) chunk = std::min<int64_t>(chunk, BIG_WG);   // one global slot per workgroup
    (void)per_chunk_cell;
    pb->chunk = (int)chunk;
    pb->lam_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nc * nn + 255) / 256));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    auto &f = pb->off;
    f.tab = take(sizeof(Tables));
    f.u0 = take(8ull * nv * nc * nn);
    f.u1 = take(8ull * nv * nc * nn);
    f.emin0 = take(8ull * nv * next);
    f.emax0 = take(8ull * nv * next);
    f.emin1 = take(8ull * nv * next);
    f.emax1 = take(8ull * nv * next);
    f.trace = take(8ull * nc * 2 * d * nv * nfn * n);
    f.gbar = take(8ull * nc * 2 * d * nv * nfn);
    f.beta0 = take(nc);
    f.beta1 = take(nc);
    f.force = take(nc);
    f.mflag = take(pb->prm.mood ? pb->cap * nsub : 1);
    f.margin = take(4ull * nc);
    f.tlist = take(4ull * nc);
    f.clist = take(4ull * nc);
    f.slot0 = take(4ull * nc);
    f.slot1 = take(4ull * nc);
    f.pool0 = take(8ull * pb->cap * nv * nsub);
    f.pool1 = take(8ull * pb->cap * nv * nsub);
    f.sflux = take(8ull * pb->cap * 2 * d * nv * nfn);
    f.blk = take(4ull * 2 * nblk);
    f.counts = take(4ull * 8);
    f.scal = take(8ull * 8);
    f.lampart = take(8ull * 1024);
    {
        int64_t inner = 1;
        for (int j = 0; j < d; j++) inner *= P.nc[j];
        pb->ring_cap = next - inner + nc;
    }
    f.ring = take(8ull * std::max<int64_t>(1, pb->ring_cap));
    f.halo = take(8ull * chunk * nv * hsz);
    f.Y = take(8ull * chunk * pb->npos * nv * n3);
    f.strace = take(8ull * chunk * pb->npos * 2 * d * nv * nf3 * 3);
    f.fpts = take(8ull * chunk * 2 * d * nv * ipow64(3 * Ns, d - 1));
    f.mask = take(nc);
    // large cells: one global slot per workgroup of their corrector, bounds, subcell and
    // flux-correction launches
    f.big = take(8ull * BIG_WG * std::max<int64_t>(1, big_slot_doubles(d, P.N)));
    f.end = o;
    pb->ws_bytes = o;
}

static void carve(adg_problem *pb) {
    char *w = pb->ws;
    auto &f = pb->off;
    Bufs &B = pb->B;
    B.tab = (Tables *)(w + f.tab);
    B.u[0] = (double *)(w + f.u0);
    B.u[1] = (double *)(w + f.u1);
    B.ext_min[0] = (double *)(w + f.emin0);
    B.ext_max[0] = (double *)(w + f.emax0);
    B.ext_min[1] = (double *)(w + f.emin1);
    B.ext_max[1] = (double *)(w + f.emax1);
    B.trace = (double *)(w + f.trace);
    B.gbar = (double *)(w + f.gbar);
    B.beta[0] = (uint8_t *)(w + f.beta0);
    B.beta[1] = (uint8_t *)(w + f.beta1);
    B.force = (uint8_t *)(w + f.force);
    B.mflag = (uint8_t *)(w + f.mflag);
    B.margin = (float *)(w + f.margin);
    B.tlist = (int *)(w + f.tlist);
    B.clist = (int *)(w + f.clist);
    B.slot[0] = (int *)(w + f.slot0);
    B.slot[1] = (int *)(w + f.slot1);
    B.pool[0] = (double *)(w + f.pool0);
    B.pool[1] = (double *)(w + f.pool1);
    B.sflux = (double *)(w + f.sflux);
    B.blk = (int *)(w + f.blk);
    B.counts = (int *)(w + f.counts);
    B.scal = (double *)(w + f.scal);
    B.lam_part = (double *)(w + f.lampart);
    B.ring = (int64_t *)(w + f.ring);
    B.halo = (double *)(w + f.halo);
    B.Y = (double *)(w + f.Y);
    B.strace = (double *)(w + f.strace);
    B.fpts = (double *)(w + f.fpts);
    B.mask = pb->mask.empty() ? nullptr : (const uint8_t *)(w + f.mask);
    B.big = (double *)(w + f.big);
    pb->tab_dev = B.tab;
}

// The masked geometry (if any) into the workspace, then the extended-grid cells whose
// old-time bounds each step computes, x fastest: the ghost-ring cells the detection reads
// (a ring cell whose out-of-range coordinates all lie on non-periodic axes; along a periodic
// axis the detection wraps to the interior cell instead), then the solid cells (their
// bounds are those of their mirror image, which the fluid's new data changes every step).
static int upload_mask_ring(adg_problem *pb) {
    const Prob &P = pb->P;
    std::vector<int64_t> ring;
    ring.reserve(pb->ring_cap);
    const int64_t ne0 = P.nc[0] + 2, ne1 = P.dim > 1 ? P.nc[1] + 2 : 1, ne2 = P.dim > 2 ? P.nc[2] + 2 : 1;
    for (int64_t k = 0; k < ne2; k++)
        for (int64_t j = 0; j < ne1; j++)
            for (int64_t i = 0; i < ne0; i++) {
                const int64_t e[3] = {i, j, k}, ne[3] = {ne0, ne1, ne2};
                bool ghost = false, periodic_image = false;
                for (int a = 0; a < P.dim; a++)
                    if (e[a] == 0 || e[a] == ne[a] - 1) {
                        ghost = true;
                        if (P.periodic[a]) periodic_image = true;
                    }
                if (ghost && !periodic_image) ring.push_back(i + ne0 * (j + ne1 * k));
            }
    if (!pb->mask.empty()) {
        for (int64_t c = 0; c < P.ncell; c++) {
            if (!pb->mask[c]) continue;
            const int64_t i = c % P.nc[0], j = P.dim > 1 ? (c / P.nc[0]) % P.nc[1] : 0,
                          k = P.dim > 2 ? c / ((int64_t)P.nc[0] * P.nc[1]) : 0;
            ring.push_back((i + 1) + ne0 * ((P.dim > 1 ? j + 1 : 0) + ne1 * (P.dim > 2 ? k + 1 : 0)));
        }
        HIPCHK(hipMemcpyAsync(pb->ws + pb->off.mask, pb->mask.data(), P.ncell, hipMemcpyHostToDevice, pb->stream));
    }
    if ((int64_t)ring.size() > pb->ring_cap) return fail(ADG_EINVAL, "internal: ghost ring size");
    pb->nring = (int64_t)ring.size();
    if (pb->nring) HIPCHK(hipMemcpyAsync(pb->B.ring, ring.data(), 8 * ring.size(), hipMemcpyHostToDevice, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    return ADG_OK;
}

static StepCtx ctx(const adg_problem *pb) {
    StepCtx C;
    C.P = pb->P;
    C.B = pb->B;
    C.tab = pb->tab_dev;
    C.stream = pb->stream;
    C.cur = pb->cur;
    C.limiter = pb->prm.limiter;
    C.picard_iters = pb->prm.picard_iters;
    C.capacity = pb->cap;
    C.lam_blocks = pb->lam_blocks;
    C.precision = pb->prm.precision;
    C.mood = pb->prm.mood;
    C.ring_only = pb->bounds_valid ? 1 : 0;
    C.subcell_grid = pb->chunk;
    C.nring = pb->nring;
    return C;
}

extern "C" {

const char *adg_last_error(void) { return g_err.c_str(); }

int adg_create(const adg_grid_desc *g, int N, double gamma, const adg_params *p, adg_problem **out) {
    if (!g || !out) return fail(ADG_EINVAL, "null argument");
    *out = nullptr;
    if (g->dim != 2 && g->dim != 3) return fail(ADG_EINVAL, "dim must be 2 or 3");
    if (!supported(g->dim, N)) return fail(ADG_EINVAL, "N=%d not built for dim=%d", N, g->dim);
    if (!(gamma > 1.0)) return fail(ADG_EINVAL, "gamma must exceed 1");
    adg_params prm{};
    if (p) prm = *p;
    else prm.limiter = 1;
    if (prm.Ns == 0) prm.Ns = 2 * N + 1;
    if (prm.Ns != 2 * N + 1)
        return fail(ADG_EINVAL, "Ns = %d: the kernels are built for Ns = 2N+1 = %d only (Sec. 4.5's choice, stable "
                    "at the DG time step of eq. (cfl)); Ns >= N+1 is not built", prm.Ns, 2 * N + 1);
    if (prm.picard_iters <= 0) prm.picard_iters = N + 1;
    if (prm.eps == 0) prm.eps = 1e-3;
    if (prm.delta0 == 0) prm.delta0 = 1e-4;
    if (prm.precision != ADG_FP64 && prm.precision != ADG_MIXED && prm.precision != ADG_MIXED_DEV)
        return fail(ADG_EINVAL, "unknown precision mode");
    if (prm.precision == ADG_MIXED_DEV && prm.flux != 0)
        return fail(ADG_EINVAL, "the deviation form is built for the Rusanov flux only");
    if (prm.mood != 0 && prm.mood != 1) return fail(ADG_EINVAL, "mood must be 0 or 1");
    if (prm.flux != 0 && prm.flux != 1) return fail(ADG_EINVAL, "flux must be 0 (Rusanov) or 1 (Osher-type)");
    adg_problem *pb = new (std::nothrow) adg_problem();
    if (!pb) return fail(ADG_ENOMEM, "host allocation failed");
    Prob &P = pb->P;
    std::memset(&P, 0, sizeof P);
    P.dim = g->dim;
    P.N = N;
    P.n = N + 1;
    P.nv = g->dim + 2;
    P.Ns = prm.Ns;
    P.ncell = 1;
    for (int k = 0; k < 3; k++) {
        if (k < g->dim) {
            if (g->n[k] < 1 || g->n[k] > (1 << 30) || !(g->hi[k] > g->lo[k])) {
                delete pb;
                return fail(ADG_EINVAL, "bad extent on axis %d", k);
            }
            P.nc[k] = (int)g->n[k];
            P.lo[k] = g->lo[k];
            P.h[k] = (g->hi[k] - g->lo[k]) / g->n[k];
        } else {
            P.nc[k] = 1;
            P.lo[k] = 0;
            P.h[k] = 1;
        }
        P.ncell *= P.nc[k];
    }
    if (P.ncell > (int64_t)1 << 31) {
        delete pb;
        return fail(ADG_EINVAL, "too many cells");
    }
    P.gamma = gamma;
    P.eps = prm.eps;
    P.flux = prm.flux;
    P.delta0 = prm.delta0;
    for (int k = 0; k < g->dim; k++) {
        const int p0 = g->bc[k][0].kind[0] == ADG_PERIODIC, p1 = g->bc[k][1].kind[0] == ADG_PERIODIC;
        if (p0 != p1) {
            delete pb;
            return fail(ADG_EINVAL, "periodic must be set on both sides of axis %d", k);
        }
        P.periodic[k] = p0;
        for (int s = 0; s < 2; s++) {
            const adg_bc &b = g->bc[k][s];
            BCDev &d = P.bc[k][s];
            for (int w = 0; w < 2; w++) {
                if (b.kind[w] < 0 || b.kind[w] > ADG_DIRICHLET) {
                    delete pb;
                    return fail(ADG_EINVAL, "bad boundary kind");
                }
                d.kind[w] = b.kind[w];
                for (int v = 0; v < 5; v++) d.state[w][v] = b.state[w][v];
            }
            if (b.split_axis >= g->dim || b.split_axis == k) {
                delete pb;
                return fail(ADG_EINVAL, "split axis must be a tangential axis");
            }
            d.split_axis = b.split_axis < 0 ? -1 : b.split_axis;
            d.split0 = b.split0;
            d.split_speed = b.split_speed;
        }
    }
    pb->prm = prm;
    pb->cap = prm.pool_capacity > 0 ? std::min<int64_t>(prm.pool_capacity, P.ncell) : P.ncell;
    pb->npos = positions_per_cell(P.dim, N);
    build_tables(N, P.Ns, &pb->tab_host);
    plan(pb);
    *out = pb;
    return ADG_OK;
}

int adg_destroy(adg_problem *pb) {
    if (!pb) return ADG_OK;
    if (pb->stream || pb->bound) (void)hipStreamSynchronize(pb->stream);
    for (auto &m : pb->pending) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (auto e : pb->spare) (void)hipEventDestroy(e);
    if (pb->counts_ready) (void)hipEventDestroy(pb->counts_ready);
    if (pb->pinned) (void)hipHostFree(pb->pinned);
    delete pb;
    return ADG_OK;
}

size_t adg_workspace_bytes(const adg_problem *pb) { return pb ? pb->ws_bytes : 0; }

int adg_bind(adg_problem *pb, void *dev_workspace, size_t bytes, void *hip_stream) {
    if (!pb || !dev_workspace) return fail(ADG_EINVAL, "null argument");
    if (bytes < pb->ws_bytes) return fail(ADG_ENOMEM, "workspace %zu bytes < %zu needed", bytes, pb->ws_bytes);
    if (((uintptr_t)dev_workspace) & 255) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
    pb->ws = (char *)dev_workspace;
    pb->stream = (hipStream_t)hip_stream;
    carve(pb);
    if (!pb->pinned) HIPCHK(hipHostMalloc((void **)&pb->pinned, 64, hipHostMallocDefault));
    HIPCHK(hipMemcpyAsync(pb->tab_dev, &pb->tab_host, sizeof(Tables), hipMemcpyHostToDevice, pb->stream));
    {
        const int rc = upload_mask_ring(pb);
        if (rc != ADG_OK) return rc;
        HIPCHK(hipStreamSynchronize(pb->stream));
    }
    HIPCHK(hipMemsetAsync(pb->B.counts, 0, 32, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.scal, 0, 64, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.force, 0, pb->P.ncell, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.beta[0], 0, pb->P.ncell, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.beta[1], 0, pb->P.ncell, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.margin, 0, 4 * pb->P.ncell, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    pb->bound = true;
    pb->has_state = false;
    pb->cur = 0;
    return ADG_OK;
}

int adg_set_mask(adg_problem *pb, const uint8_t *mask) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (pb->batch) return fail(ADG_ESTATE, "the problem belongs to a batch: destroy the batch first");
    const Prob &P = pb->P;
    pb->mask.clear();
    if (mask) {
        int64_t nsolid = 0;
        pb->mask.assign(P.ncell, 0);
        for (int64_t c = 0; c < P.ncell; c++) {
            pb->mask[c] = mask[c] ? 1 : 0;
            nsolid += pb->mask[c];
        }
        if (nsolid == P.ncell) {
            pb->mask.clear();
            return fail(ADG_EINVAL, "every cell is solid");
        }
        if (nsolid == 0) pb->mask.clear();
    }
    if (!pb->bound) return ADG_OK;
    pb->B.mask = pb->mask.empty() ? nullptr : (const uint8_t *)(pb->ws + pb->off.mask);
    pb->bounds_valid = false;   // solid cells' old-time bounds are computed by the next step
    return upload_mask_ring(pb);
}

int adg_axis_points(const adg_problem *pb, int axis, int m, double *out) {
    if (!pb || !out || axis < 0 || axis >= pb->P.dim || m < 0 || m > 16) return fail(ADG_EINVAL, "bad argument");
    const Prob &P = pb->P;
    if (m == 0) {
        for (int i = 0; i < P.nc[axis]; i++)
            for (int a = 0; a < P.n; a++) out[(int64_t)i * P.n + a] = P.lo[axis] + P.h[axis] * (i + pb->tab_host.xi[a]);
        return ADG_OK;
    }
    double xq[16], wq[16];
    gl_nodes(m, xq, wq);
    for (int i = 0; i < P.nc[axis]; i++)
        for (int s = 0; s < P.Ns; s++)
            for (int q = 0; q < m; q++)
                out[((int64_t)i * P.Ns + s) * m + q] = P.lo[axis] + P.h[axis] * (i + (s + xq[q]) / P.Ns);
    return ADG_OK;
}

// out = (M x M (x M)) in: M is mo x mi with row stride ld, in holds mi^d values (x fastest),
// out mo^d; applied axis by axis (sum factorisation), t1 / t2 hold the intermediate stages.
static void tensor_host(int d, int mo, int mi, const double *M, int ld, const double *in, double *out,
                        std::vector<double> &t1, std::vector<double> &t2) {
    int dims[3] = {mi, mi, mi};
    const double *src = in;
    for (int k = 0; k < d; k++) {
        int dn[3] = {dims[0], dims[1], dims[2]};
        dn[k] = mo;
        int64_t tot = 1, stride = 1;
        for (int j = 0; j < d; j++) tot *= dn[j];
        for (int j = 0; j < k; j++) stride *= dims[j];
        std::vector<double> &buf = (k % 2 == 0) ? t1 : t2;
        if (k < d - 1 && (int64_t)buf.size() < tot) buf.resize(tot);
        double *dst = (k == d - 1) ? out : buf.data();
        for (int64_t e = 0; e < tot; e++) {
            int mm[3] = {0, 0, 0};
            int64_t r = e, base = 0, mul = 1;
            for (int j = 0; j < d; j++) {
                mm[j] = (int)(r % dn[j]);
                r /= dn[j];
            }
            for (int j = 0; j < d; j++) {
                if (j != k) base += mm[j] * mul;
                mul *= dims[j];
            }
            const double *row = M + (int64_t)mm[k] * ld;
            double acc = 0.0;
            for (int b = 0; b < mi; b++) acc += row[b] * src[base + b * stride];
            dst[e] = acc;
        }
        dims[k] = mo;
        src = dst;
    }
}

int adg_project_samples(const adg_problem *pb, const double *samples, int m, double *u, double *v) {
    if (!pb || !samples || !u || m < 0 || m > 16) return fail(ADG_EINVAL, "bad argument");
    const Prob &P = pb->P;
    const int d = P.dim, n = P.n, Ns = P.Ns, nv = P.nv;
    const int64_t nn = ipow64(n, d), nsub = ipow64(Ns, d), nc = P.ncell;
    const int per = m == 0 ? n : Ns * m;
    int64_t ext[3] = {1, 1, 1};
    for (int k = 0; k < d; k++) ext[k] = (int64_t)P.nc[k] * per;
    const int64_t npts = ext[0] * ext[1] * ext[2];
    if (m == 0) {
        parallel_for(nc, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; c++) {
                int ci[3] = {(int)(c % P.nc[0]), (int)((c / P.nc[0]) % P.nc[1]), (int)(c / ((int64_t)P.nc[0] * P.nc[1]))};
                for (int64_t a = 0; a < nn; a++) {
                    int ma[3] = {(int)(a % n), (int)((a / n) % n), (int)(a / (n * n))};
                    int64_t gi[3] = {0, 0, 0};
                    for (int k = 0; k < d; k++) gi[k] = (int64_t)ci[k] * per + ma[k];
                    const int64_t pidx = gi[0] + ext[0] * (gi[1] + ext[1] * gi[2]);
                    for (int vv = 0; vv < nv; vv++) u[((int64_t)vv * nc + c) * nn + a] = samples[vv * npts + pidx];
                }
            }
        });
        return ADG_OK;
    }
    // composite m-point rule on every subcell.  u: the L2 projection onto the nodal basis,
    // u_a = sum over points of w * phi_a * f / (w_a Ns^d) (mass matrix diagonal in the GL
    // nodal basis), applied axis by axis with the per-axis matrix w_q phi_a(x_q); v: the
    // rule's subcell averages.
    double xq[16], wq[16];
    gl_nodes(m, xq, wq);
    const int pa = Ns * m;   // points per axis and cell
    std::vector<double> phw((size_t)n * pa), phi(n);
    for (int s = 0; s < Ns; s++)
        for (int q = 0; q < m; q++) {
            lagrange_values(n, pb->tab_host.xi, (s + xq[q]) / Ns, phi.data());
            for (int a = 0; a < n; a++) phw[(size_t)a * pa + s * m + q] = wq[q] * phi[a];
        }
    const int64_t nq = ipow64(m, d), npc = ipow64(pa, d);
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
        std::vector<double> f((size_t)npc), out((size_t)nn), t1, t2;
        for (int64_t c = c0; c < c1; c++) {
            int ci[3] = {(int)(c % P.nc[0]), (int)((c / P.nc[0]) % P.nc[1]), (int)(c / ((int64_t)P.nc[0] * P.nc[1]))};
            for (int vv = 0; vv < nv; vv++) {
                // the cell's points, x fastest
                for (int64_t e = 0; e < npc; e++) {
                    const int64_t me[3] = {e % pa, (e / pa) % pa, e / ((int64_t)pa * pa)};
                    int64_t gi[3] = {0, 0, 0};
                    for (int k = 0; k < d; k++) gi[k] = (int64_t)ci[k] * pa + me[k];
                    f[e] = samples[vv * npts + gi[0] + ext[0] * (gi[1] + ext[1] * gi[2])];
                }
                if (v)
                    for (int64_t sg = 0; sg < nsub; sg++) {
                        const int ms[3] = {(int)(sg % Ns), (int)((sg / Ns) % Ns), (int)(sg / (Ns * Ns))};
                        double avg = 0.0;
                        for (int64_t qi = 0; qi < nq; qi++) {
                            const int mq[3] = {(int)(qi % m), (int)((qi / m) % m), (int)(qi / (m * m))};
                            double w = 1.0;
                            int64_t e = 0;
                            for (int k = d - 1; k >= 0; k--) {
                                w *= wq[mq[k]];
                                e = e * pa + ms[k] * m + mq[k];
                            }
                            avg += w * f[e];
                        }
                        v[((int64_t)vv * nc + c) * nsub + sg] = avg;
                    }
                tensor_host(d, n, pa, phw.data(), pa, f.data(), out.data(), t1, t2);
                for (int64_t a = 0; a < nn; a++) {
                    const int ma[3] = {(int)(a % n), (int)((a / n) % n), (int)(a / (n * n))};
                    double W = 1.0;
                    for (int k = 0; k < d; k++) W *= pb->tab_host.w[ma[k]];
                    u[((int64_t)vv * nc + c) * nn + a] = out[a] / (W * nsub);
                }
            }
        }
    });
    return ADG_OK;
}

// Host-side initial detection (Sec. 4.4, last paragraph): P(u0) against the bounds of
// the exact subcell averages over each cell's neighbourhood.
static int initial_detection(adg_problem *pb, std::vector<double> &u, const double *vex, std::vector<uint8_t> &beta,
                             std::vector<int> &slot, std::vector<double> &pool, int64_t &count) {
    const Prob &P = pb->P;
    const Tables &T = pb->tab_host;
    const int d = P.dim, n = P.n, Ns = P.Ns, nv = P.nv;
    const int64_t nn = ipow64(n, d), nsub = ipow64(Ns, d), nc = P.ncell;
    beta.assign(nc, 0);
    slot.assign(nc, -1);
    count = 0;
    // value of one subcell of a ghost cell (outside a non-periodic side): the boundary rule
    // applied to the mirrored interior subcell
    auto ghost_value = [&](const int *gci, const int *gs, double *q) {
        int src[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gside[3] = {-1, -1, -1};
        for (int j = 0; j < d; j++) {
            src[j] = gci[j];
            ss[j] = gs[j];
            if (gci[j] < 0 || gci[j] >= P.nc[j]) {
                const int side = gci[j] >= P.nc[j];
                if (P.periodic[j]) src[j] = (gci[j] + P.nc[j]) % P.nc[j];
                else {
                    src[j] = side ? 2 * P.nc[j] - 1 - gci[j] : -1 - gci[j];
                    ss[j] = Ns - 1 - gs[j];
                    gside[j] = side;
                }
            }
        }
        const int64_t cs = src[0] + (int64_t)P.nc[0] * (src[1] + (int64_t)P.nc[1] * src[2]);
        int sidx = 0;
        for (int j = d - 1; j >= 0; j--) sidx = sidx * Ns + ss[j];
        for (int vv = 0; vv < nv; vv++) q[vv] = vex[((int64_t)vv * nc + cs) * nsub + sidx];
        double x[3] = {0, 0, 0};
        for (int j = 0; j < d; j++) x[j] = P.lo[j] + P.h[j] * (gci[j] + (gs[j] + 0.5) / Ns);
        for (int j = 0; j < d; j++) {
            if (gside[j] < 0) continue;
            const BCDev &b = P.bc[j][gside[j]];
            int which = 0;
            if (b.split_axis >= 0) which = (x[b.split_axis] < b.split0) ? 0 : 1;
            if (b.kind[which] == ADG_DIRICHLET) {
                for (int vv = 0; vv < nv; vv++) q[vv] = b.state[which][vv];
            } else if (b.kind[which] == ADG_REFLECTIVE) {
                q[1 + j] = -q[1 + j];
            }
        }
    };
    // masked geometry: is the cell at global coordinates g solid (outside a periodic axis it
    // wraps, outside another it is the interior cell it mirrors)
    const uint8_t *mask = pb->mask.empty() ? nullptr : pb->mask.data();
    auto solid_at_host = [&](const int *g) -> bool {
        if (!mask) return false;
        int64_t cc = 0;
        for (int j = d - 1; j >= 0; j--) {
            const int nk = P.nc[j];
            int x = g[j];
            if (x < 0 || x >= nk) x = P.periodic[j] ? ((x % nk) + nk) % nk : (x >= nk ? 2 * nk - 1 - x : -1 - x);
            cc = cc * nk + x;
        }
        return mask[cc] != 0;
    };
    // value of one subcell of any cell: a solid cell holds the mirror image of the fluid
    // across its walls (the lower fluid face neighbour along an axis first, else the upper;
    // the subcell index reversed and the momentum negated along every mirrored axis)
    auto sub_value = [&](const int *gci_in, const int *gs_in, double *q) {
        int gci[3] = {gci_in[0], gci_in[1], gci_in[2]}, gs[3] = {gs_in[0], gs_in[1], gs_in[2]};
        int istep[3] = {0, 0, 0};
        if (solid_at_host(gci)) {
            for (int k = 0; k < d; k++) {
                int lo[3] = {gci[0], gci[1], gci[2]}, hi[3] = {gci[0], gci[1], gci[2]};
                lo[k] -= 1;
                hi[k] += 1;
                istep[k] = !solid_at_host(lo) ? -1 : (!solid_at_host(hi) ? 1 : 0);
            }
            for (int k = 0; k < d; k++)
                if (istep[k]) {
                    gci[k] += istep[k];
                    gs[k] = Ns - 1 - gs[k];
                }
        }
        ghost_value(gci, gs, q);
        for (int k = 0; k < d; k++)
            if (istep[k]) q[1 + k] = -q[1 + k];
    };
    // per-cell extrema of the exact subcell data
    std::vector<double> cmin((size_t)nc * nv), cmax((size_t)nc * nv);
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; c++)
            for (int vv = 0; vv < nv; vv++) {
                double lo = INFINITY, hi = -INFINITY;
                const double *x = vex + ((int64_t)vv * nc + c) * nsub;
                for (int64_t sg = 0; sg < nsub; sg++) {
                    lo = std::fmin(lo, x[sg]);
                    hi = std::fmax(hi, x[sg]);
                }
                cmin[(size_t)c * nv + vv] = lo;
                cmax[(size_t)c * nv + vv] = hi;
            }
    });
    std::vector<uint8_t> flag(nc, 0);
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
        std::vector<double> vstar((size_t)nsub), t1, t2;
        std::vector<double> vs((size_t)nv * nsub);
        for (int64_t c = c0; c < c1; c++) {
            if (mask && mask[c]) continue;   // solid cells are never troubled
            int ci[3] = {(int)(c % P.nc[0]), (int)((c / P.nc[0]) % P.nc[1]), (int)(c / ((int64_t)P.nc[0] * P.nc[1]))};
            double lo[5], hi[5];
            for (int vv = 0; vv < nv; vv++) {
                lo[vv] = INFINITY;
                hi[vv] = -INFINITY;
            }
            // bounds over the 3^d neighbourhood: stored extrema of interior (or periodically
            // wrapped) fluid cells, subcell by subcell for ghost and solid cells
            const int nb = (int)ipow64(3, d);
            for (int o = 0; o < nb; o++) {
                int gci[3] = {ci[0], ci[1], ci[2]};
                const int off[3] = {o % 3, (o / 3) % 3, o / 9};
                bool ghost = false;
                int src[3] = {0, 0, 0};
                for (int j = 0; j < d; j++) {
                    gci[j] += off[j] - 1;
                    src[j] = gci[j];
                    if (gci[j] < 0 || gci[j] >= P.nc[j]) {
                        if (P.periodic[j]) src[j] = (gci[j] + P.nc[j]) % P.nc[j];
                        else ghost = true;
                    }
                }
                if (!ghost && !solid_at_host(gci)) {
                    const int64_t cs = src[0] + (int64_t)P.nc[0] * (src[1] + (int64_t)P.nc[1] * src[2]);
                    for (int vv = 0; vv < nv; vv++) {
                        lo[vv] = std::fmin(lo[vv], cmin[(size_t)cs * nv + vv]);
                        hi[vv] = std::fmax(hi[vv], cmax[(size_t)cs * nv + vv]);
                    }
                    continue;
                }
                for (int64_t sg = 0; sg < nsub; sg++) {
                    const int gs[3] = {(int)(sg % Ns), (int)((sg / Ns) % Ns), (int)(sg / (Ns * Ns))};
                    double q[5];
                    sub_value(gci, gs, q);
                    for (int vv = 0; vv < nv; vv++) {
                        lo[vv] = std::fmin(lo[vv], q[vv]);
                        hi[vv] = std::fmax(hi[vv], q[vv]);
                    }
                }
            }
            // candidate subcell averages P(u0)
            for (int vv = 0; vv < nv; vv++)
                tensor_host(d, Ns, n, &T.P[0][0], MAXN, &u[((int64_t)vv * nc + c) * nn], &vs[(size_t)vv * nsub], t1, t2);
            bool bad = false;
            for (int64_t sg = 0; sg < nsub && !bad; sg++) {
                double q[5];
                bool finite = true;
                for (int vv = 0; vv < nv; vv++) {
                    q[vv] = vs[(size_t)vv * nsub + sg];
                    finite = finite && std::isfinite(q[vv]);
                }
                if (!finite) {
                    bad = true;
                    break;
                }
                double ke = 0;
                for (int j = 0; j < d; j++) ke += q[1 + j] * q[1 + j];
                const double p = (P.gamma - 1.0) * (q[d + 1] - 0.5 * ke / q[0]);
                if (!(q[0] > 0) || !(p > 0)) bad = true;
                for (int vv = 0; vv < nv; vv++) {
                    const double delta = std::fmax(P.delta0, P.eps * (hi[vv] - lo[vv]));
                    if (q[vv] < lo[vv] - delta || q[vv] > hi[vv] + delta) bad = true;
                }
            }
            flag[c] = bad;
        }
    });
    // pool slots in cell order
    std::vector<int64_t> list;
    for (int64_t c = 0; c < nc; c++) {
        if (!flag[c]) continue;
        if (count >= pb->cap) return fail(ADG_ECAPACITY, "initial detection flags more cells than the pool holds");
        beta[c] = 1;
        slot[c] = (int)count;
        list.push_back(c);
        count++;
    }
    // troubled cells: the exact subcell data into the pool, u := R(v_exact)
    pool.assign((size_t)count * nv * nsub, 0.0);
    parallel_for(count, [&](int64_t i0, int64_t i1) {
        std::vector<double> t1, t2;
        for (int64_t i = i0; i < i1; i++) {
            const int64_t c = list[i];
            for (int vv = 0; vv < nv; vv++) {
                const double *vc = vex + ((int64_t)vv * nc + c) * nsub;
                std::copy(vc, vc + nsub, pool.begin() + ((size_t)i * nv + vv) * nsub);
                tensor_host(d, n, Ns, &T.Rg[0][0], MAXNS, vc, &u[((int64_t)vv * nc + c) * nn], t1, t2);
            }
        }
    });
    return ADG_OK;
}

int adg_set_state(adg_problem *pb, const double *u, int on_device, const double *v_exact) {
    if (!pb || !u) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "adg_bind first");
    if (pb->batch) return fail(ADG_ESTATE, "the problem belongs to a batch: destroy the batch first");
    const Prob &P = pb->P;
    const int64_t nn = ipow64(P.n, P.dim), nsub = ipow64(P.Ns, P.dim);
    const size_t ubytes = 8ull * P.nv * P.ncell * nn;
    pb->cur = 0;
    std::vector<uint8_t> beta(P.ncell, 0);
    std::vector<int> slot(P.ncell, -1);
    int64_t count = 0;
    if (v_exact && pb->prm.limiter) {
        std::vector<double> uh((size_t)P.nv * P.ncell * nn);
        if (on_device) {
            HIPCHK(hipMemcpyAsync(uh.data(), u, ubytes, hipMemcpyDeviceToHost, pb->stream));
            HIPCHK(hipStreamSynchronize(pb->stream));
        } else {
            std::memcpy(uh.data(), u, ubytes);
        }
        std::vector<double> pool;
        int rc = initial_detection(pb, uh, v_exact, beta, slot, pool, count);
        if (rc != ADG_OK) return rc;
        HIPCHK(hipMemcpyAsync(pb->B.u[0], uh.data(), ubytes, hipMemcpyHostToDevice, pb->stream));
        if (count)
            HIPCHK(hipMemcpyAsync(pb->B.pool[0], pool.data(), 8ull * count * P.nv * nsub, hipMemcpyHostToDevice,
                                  pb->stream));
        HIPCHK(hipStreamSynchronize(pb->stream));
    } else {
        HIPCHK(hipMemcpyAsync(pb->B.u[0], u, ubytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              pb->stream));
    }
    HIPCHK(hipMemcpyAsync(pb->B.beta[0], beta.data(), P.ncell, hipMemcpyHostToDevice, pb->stream));
    HIPCHK(hipMemcpyAsync(pb->B.slot[0], slot.data(), 4ull * P.ncell, hipMemcpyHostToDevice, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.scal, 0, 64, pb->stream));
    HIPCHK(hipMemsetAsync(pb->B.counts, 0, 32, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    // the host copy of the counters starts over too (a pool overflow is reported until here)
    std::memset(pb->pinned, 0, 16);
    pb->nonphys_reported = 0;
    pb->has_state = true;
    pb->bounds_valid = false;
    pb->last_troubled = count;
    pb->last_corrected = 0;
    pb->steps = 0;
    return ADG_OK;
}

int adg_state_device_ptr(const adg_problem *pb, const double **u) {
    if (!pb || !u) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    *u = pb->B.u[pb->cur];
    return ADG_OK;
}

int adg_get_state(const adg_problem *pb, double *u, int to_device) {
    if (!pb || !u) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    const size_t ubytes = 8ull * pb->P.nv * pb->P.ncell * ipow64(pb->P.n, pb->P.dim);
    HIPCHK(hipMemcpyAsync(u, pb->B.u[pb->cur], ubytes, to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          pb->stream));
    if (!to_device) HIPCHK(hipStreamSynchronize(pb->stream));
    return ADG_OK;
}

static double dt_factor(const adg_problem *pb, double cfl) {
    double h = pb->P.h[0];
    for (int k = 1; k < pb->P.dim; k++) h = std::fmin(h, pb->P.h[k]);
    return cfl * h / (pb->P.dim * (2.0 * pb->P.N + 1.0));
}

int adg_cfl_dt(adg_problem *pb, double cfl, double *dt_out) {
    if (!pb || !dt_out || !(cfl > 0)) return fail(ADG_EINVAL, "bad argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    StepCtx C = ctx(pb);
    launch_lambda(C, pb->B.u[pb->cur], dt_factor(pb, cfl));
    HIPCHK(hipGetLastError());
    double s[3];
    HIPCHK(hipMemcpyAsync(s, pb->B.scal, sizeof s, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    *dt_out = s[0];
    return ADG_OK;
}

// ADG_ENONPHYSICAL once the counter of subcell results failing PAD (copied to the host
// after every step) has risen since the last report; ADG_OK otherwise.
static int nonphysical_news(adg_problem *pb) {
    if (pb->pinned && pb->pinned[2] > pb->nonphys_reported) {
        const int64_t now = pb->pinned[2];
        const int rc = fail(ADG_ENONPHYSICAL, "%lld subcell results failed positivity so far (%lld new)",
                            (long long)now, (long long)(now - pb->nonphys_reported));
        pb->nonphys_reported = now;
        return rc;
    }
    return ADG_OK;
}

static int do_step(adg_problem *pb) {
    StepCtx C = ctx(pb);
    Bufs &B = pb->B;
    if (!pb->capturing && pb->counts_ready && hipEventQuery(pb->counts_ready) == hipSuccess && pb->pinned[3])
        return fail(ADG_ECAPACITY, "troubled cells exceeded the pool capacity %lld in an earlier step",
                    (long long)pb->cap);
    const int news = (!pb->capturing && pb->counts_ready && hipEventQuery(pb->counts_ready) == hipSuccess)
                         ? nonphysical_news(pb) : ADG_OK;
    if (pb->prm.limiter) {
        GroupTimer g(pb, 0);
        launch_bounds(C);
    }
    {
        GroupTimer g(pb, 1);
        launch_predictor(C);
    }
    {
        GroupTimer g(pb, 2);
        launch_faces(C);
    }
    {
        GroupTimer g(pb, 3);
        launch_corrector_detect(C);
    }
    HIPCHK(hipGetLastError());
    int64_t troubled = 0, corrected = 0;
    int rc = ADG_OK;
    if (pb->prm.limiter) {
        {
            GroupTimer g(pb, 4);
            launch_compact(C);
        }
        HIPCHK(hipGetLastError());
        // no host wait: the subcell recompute and the flux correction read the counts on
        // the device
        {
            GroupTimer g(pb, 5);
            launch_subcell(C, 0);
            if (pb->prm.mood) launch_subcell(C, 1);   // the MOOD layer's recompute
        }
        {
            GroupTimer g(pb, 6);
            launch_fluxcorr(C, -1, 1);
        }
        troubled = corrected = -1;
        HIPCHK(hipGetLastError());
        std::swap(B.beta[0], B.beta[1]);
        std::swap(B.slot[0], B.slot[1]);
        std::swap(B.pool[0], B.pool[1]);
        std::swap(B.ext_min[0], B.ext_min[1]);
        std::swap(B.ext_max[0], B.ext_max[1]);
        // every interior cell's next old-time bounds were written by this step's kernels
        pb->bounds_valid = true;
    }
    if (!pb->prm.limiter) launch_advance_time(C);   // else done by the flux correction
    HIPCHK(hipGetLastError());
    if (pb->prm.limiter && troubled < 0 && !pb->capturing) {
        // asynchronous copy of the counters (read by adg_get_stats and the next step)
        HIPCHK(hipMemcpyAsync(pb->pinned, B.counts, 16, hipMemcpyDeviceToHost, pb->stream));
        if (!pb->counts_ready) HIPCHK(hipEventCreateWithFlags(&pb->counts_ready, hipEventDisableTiming));
        HIPCHK(hipEventRecord(pb->counts_ready, pb->stream));
    }
    pb->cur ^= 1;
    pb->last_troubled = troubled;
    pb->last_corrected = corrected;
    pb->steps++;
    return rc != ADG_OK ? rc : news;
}

static int in_foreign_batch(const adg_problem *pb) {
    return pb->batch && !pb->batch_driving;
}

int adg_step(adg_problem *pb, double dt) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    if (in_foreign_batch(pb)) return fail(ADG_ESTATE, "the problem belongs to a batch: step it with adg_batch_step_cfl");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(ADG_EINVAL, "dt must be positive");
    StepCtx C = ctx(pb);
    launch_set_scalar(C, 0, dt);
    return do_step(pb);
}

int adg_step_cfl(adg_problem *pb, double cfl) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    if (in_foreign_batch(pb)) return fail(ADG_ESTATE, "the problem belongs to a batch: step it with adg_batch_step_cfl");
    if (!(cfl > 0)) return fail(ADG_EINVAL, "cfl must be positive");
    StepCtx C = ctx(pb);
    {
        GroupTimer g(pb, 7);
        launch_lambda(C, pb->B.u[pb->cur], dt_factor(pb, cfl));
    }
    return do_step(pb);
}

int adg_time(const adg_problem *pb, double *t) {
    if (!pb || !t) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    double s[2];
    HIPCHK(hipMemcpyAsync(s, pb->B.scal, sizeof s, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    *t = s[1];
    return ADG_OK;
}

int adg_get_troubled(const adg_problem *pb, uint8_t *beta, int64_t *count) {
    if (!pb || !beta) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    HIPCHK(hipMemcpyAsync(beta, pb->B.beta[0], pb->P.ncell, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    if (count) {
        int64_t s = 0;
        for (int64_t c = 0; c < pb->P.ncell; c++) s += beta[c] != 0;
        *count = s;
    }
    return ADG_OK;
}

int adg_get_margin(const adg_problem *pb, float *margin) {
    if (!pb || !margin) return fail(ADG_EINVAL, "null argument");
    HIPCHK(hipMemcpyAsync(margin, pb->B.margin, 4ull * pb->P.ncell, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    return ADG_OK;
}

int adg_get_subcells(const adg_problem *pb, double *v) {
    if (!pb || !v) return fail(ADG_EINVAL, "null argument");
    if (!pb->has_state) return fail(ADG_ESTATE, "no state");
    const Prob &P = pb->P;
    const int64_t nsub = ipow64(P.Ns, P.dim), nc = P.ncell;
    std::vector<uint8_t> beta(nc);
    std::vector<int> slot(nc);
    HIPCHK(hipMemcpyAsync(beta.data(), pb->B.beta[0], nc, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipMemcpyAsync(slot.data(), pb->B.slot[0], 4ull * nc, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    std::vector<double> buf((size_t)P.nv * nsub);
    for (int64_t c = 0; c < nc; c++) {
        if (!beta[c] || slot[c] < 0) continue;
        HIPCHK(hipMemcpyAsync(buf.data(), pb->B.pool[0] + (size_t)slot[c] * P.nv * nsub, 8ull * P.nv * nsub,
                              hipMemcpyDeviceToHost, pb->stream));
        HIPCHK(hipStreamSynchronize(pb->stream));
        for (int vv = 0; vv < P.nv; vv++)
            std::memcpy(v + ((int64_t)vv * nc + c) * nsub, buf.data() + (size_t)vv * nsub, 8ull * nsub);
    }
    return ADG_OK;
}

int adg_get_stats(const adg_problem *pb, int64_t *out4) {
    if (!pb || !out4) return fail(ADG_EINVAL, "null argument");
    int cnt[4];
    HIPCHK(hipMemcpyAsync(cnt, pb->B.counts, sizeof cnt, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    out4[0] = pb->last_troubled >= 0 ? pb->last_troubled : cnt[0];
    out4[1] = pb->last_corrected >= 0 ? pb->last_corrected : cnt[1];
    out4[2] = cnt[2];
    out4[3] = pb->steps;
    return ADG_OK;
}

int adg_get_mood_stats(const adg_problem *pb, int64_t *flagged, int64_t *redone) {
    if (!pb || !flagged || !redone) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    int c[8];
    HIPCHK(hipMemcpyAsync(c, pb->B.counts, sizeof c, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    *flagged = c[5];
    *redone = c[6];
    return ADG_OK;
}

int adg_profile(adg_problem *pb, int enable) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    HIPCHK(hipStreamSynchronize(pb->stream));
    harvest(pb);
    if (enable) {
        for (int g = 0; g < 8; g++) {
            pb->prof_ms[g] = 0;
            pb->prof_n[g] = 0;
        }
    }
    pb->prof_mask = (unsigned)enable & 0xFFu;
    return ADG_OK;
}

int adg_profile_read(adg_problem *pb, double *ms, int64_t *launches, int ngroups) {
    if (!pb || ngroups < 0 || ngroups > 8) return fail(ADG_EINVAL, "bad argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    HIPCHK(hipStreamSynchronize(pb->stream));
    harvest(pb);
    for (int g = 0; g < ngroups; g++) {
        if (ms) ms[g] = pb->prof_ms[g];
        if (launches) launches[g] = pb->prof_n[g];
    }
    return ADG_OK;
}

}  // extern "C"

// One (d, N) class of a batch: its problems share every kernel instantiation.
struct BatchClass {
    int dim = 0, N = 0;
    std::vector<int> members;             // indices into adg_batch::ps
    std::vector<BTile> tiles[6];          // lambda, bounds, predictor, face, corrector, compaction
    size_t off_ents[2] = {0, 0}, off_tiles[6] = {0, 0, 0, 0, 0, 0}, off_wt = 0, off_wc = 0;
    size_t off_Y = 0, off_tr = 0, off_halo = 0, off_fp = 0;
    int sub_grid = 0, fc_grid = 0;
};

struct adg_batch {
    std::vector<adg_problem *> ps;
    std::vector<BatchClass> cls;
    std::vector<hipStream_t> saved;       // the problems' own streams
    hipStream_t user = nullptr;           // the caller's stream bound to the batch
    hipStream_t stream = nullptr;         // the batch's own stream: captures and replays (a
                                          // legacy null stream cannot be captured)
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    int precision = 0, limiter = 1, mood = 0;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    int parity = 0;                       // which graph advances the current state
    bool captured = false;
    double cfl = 0;
    // stage timing: events at the start of every stage and at the end, inside the graphs
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> ev[2];        // [stage * nclass + class], then one at the end
    bool ev_pending[2] = {false, false};
    std::vector<double> prof_ms;          // [stage * nclass + class] total milliseconds
    int64_t prof_n = 0;                   // timed steps
};

// Host-side bookkeeping of one step (what do_step does after its launches), for replays.
static void host_advance(adg_problem *pb) {
    Bufs &B = pb->B;
    if (pb->prm.limiter) {
        std::swap(B.beta[0], B.beta[1]);
        std::swap(B.slot[0], B.slot[1]);
        std::swap(B.pool[0], B.pool[1]);
        std::swap(B.ext_min[0], B.ext_min[1]);
        std::swap(B.ext_max[0], B.ext_max[1]);
        pb->bounds_valid = true;
    }
    pb->cur ^= 1;
    pb->last_troubled = pb->last_corrected = -1;
    pb->steps++;
}

// Layout of the batch workspace: per class, the entries of both buffer parities, the tile
// tables of the stages, the global worklist offsets and the subcell scratch slots.
static void batch_plan(adg_batch *b) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return r;
    };
    for (auto &K : b->cls) {
        const size_t np = K.members.size();
        for (int t = 0; t < 6; t++) K.tiles[t].clear();
        for (size_t q = 0; q < np; q++) {
            const adg_problem *pb = b->ps[K.members[q]];
            const Prob &P = pb->P;
            const int64_t nn = ipow64(P.n, P.dim);
            const int lam_nb = (int)std::min<int64_t>(pb->lam_blocks, (P.ncell * nn + 255) / 256);
            int64_t kb1 = 0, kb2 = 0;
            const int64_t nblk[6] = {lam_nb, b->limiter ? pb->nring : 0,
                                     stage_blocks(BSTAGE_PREDICTOR, P, b->precision, &kb1, &kb2),
                                     stage_blocks(BSTAGE_FACE, P, b->precision, &kb1, &kb2),
                                     stage_blocks(BSTAGE_CORRECTOR, P, b->precision, &kb1, &kb2),
                                     b->limiter ? stage_blocks(BSTAGE_COMPACT, P, b->precision, &kb1, &kb2) : 0};
            for (int t = 0; t < 6; t++)
                for (int64_t x = 0; x < nblk[t]; x++) K.tiles[t].push_back(BTile{(int)q, (int)x, (int)nblk[t]});
        }
        for (int g = 0; g < 2; g++) K.off_ents[g] = take(sizeof(BatchEntry) * np);
        for (int t = 0; t < 6; t++) K.off_tiles[t] = take(sizeof(BTile) * K.tiles[t].size());
        K.off_wt = take(4 * (np + 1));
        K.off_wc = take(4 * (np + 1));
        // subcell scratch: one slot per workgroup of the persistent launch (as many as the
        // chip holds at once)
        const int d = K.dim, nv = d + 2, Ns = 2 * K.N + 1;
        int64_t caps = 0;
        for (int m : K.members) caps += b->ps[m]->cap;
        K.sub_grid = (int)std::max<int64_t>(1, std::min<int64_t>(subcell_workgroups(K.dim, K.N, b->precision), caps));
        K.fc_grid = 1024;
        const int64_t npos = positions_per_cell(d, K.N), n3 = ipow64(3, d), nf3 = ipow64(3, d - 1);
        const int64_t G = K.sub_grid;
        K.off_Y = take(8ull * G * npos * nv * n3);
        K.off_tr = take(8ull * G * npos * 2 * d * nv * nf3 * 3);
        K.off_halo = take(d == 3 ? 8ull * G * nv * ipow64(Ns + 6, d) : 8);
        K.off_fp = take(8ull * G * 2 * d * nv * ipow64(3 * Ns, d - 1));
    }
    b->ws_bytes = o;
}

// The launch arguments of one problem at one buffer parity (g = 0: as the problem stands,
// g = 1: after one more step's buffer swaps).
static BatchEntry batch_entry(const adg_problem *pb, int g, double cfl, int precision) {
    Bufs B = pb->B;
    int cur = pb->cur;
    if (g == 1) {
        if (pb->prm.limiter) {
            std::swap(B.beta[0], B.beta[1]);
            std::swap(B.slot[0], B.slot[1]);
            std::swap(B.pool[0], B.pool[1]);
            std::swap(B.ext_min[0], B.ext_min[1]);
            std::swap(B.ext_max[0], B.ext_max[1]);
        }
        cur ^= 1;
    }
    BatchEntry e;
    std::memset((void *)&e, 0, sizeof e);
    e.T = pb->tab_dev;
    e.P = pb->P;
    e.B = B;
    e.cur = cur;
    e.limiter = pb->prm.limiter;
    e.cap = pb->cap;
    int64_t kb1 = 0, kb2 = 0;
    (void)stage_blocks(BSTAGE_FACE, pb->P, precision, &kb1, &kb2);
    e.kb1 = kb1;
    e.kb2 = kb2;
    const int64_t nn = ipow64(pb->P.n, pb->P.dim);
    e.lam_nb = (int)std::min<int64_t>(pb->lam_blocks, (pb->P.ncell * nn + 255) / 256);
    e.factor = dt_factor(pb, cfl);
    e.ring = B.ring;
    StepCtx C = ctx(pb);
    C.B = B;
    C.cur = cur;
    predictor_args(C, &e.pf, &e.pd);
    return e;
}

static BatchLaunch batch_launch(const adg_batch *b, const BatchClass &K, int g) {
    BatchLaunch L;
    std::memset((void *)&L, 0, sizeof L);
    char *w = b->ws;
    L.E = (const BatchEntry *)(w + K.off_ents[g]);
    L.np = (int)K.members.size();
    // every member of a class has the same (d, N) and Ns = 2N+1, so the same tables: the
    // first member's copy serves the class, passed as a kernel argument (read through
    // scalar loads, like the per-problem kernels' tables)
    L.T = b->ps[K.members[0]]->tab_dev;
    const BTile **tp[6] = {&L.t_lambda, &L.t_bounds, &L.t_pred, &L.t_face, &L.t_corr, &L.t_compact};
    int *np_[6] = {&L.n_lambda, &L.n_bounds, &L.n_pred, &L.n_face, &L.n_corr, &L.n_compact};
    for (int t = 0; t < 6; t++) {
        *tp[t] = (const BTile *)(w + K.off_tiles[t]);
        *np_[t] = (int)K.tiles[t].size();
    }
    L.off_t = (int *)(w + K.off_wt);
    L.off_c = (int *)(w + K.off_wc);
    L.S = SubScratch{(double *)(w + K.off_Y), (double *)(w + K.off_tr), (double *)(w + K.off_halo),
                     (double *)(w + K.off_fp)};
    L.sub_grid = K.sub_grid;
    L.fc_grid = K.fc_grid;
    L.precision = b->precision;
    L.mood = b->mood;
    L.stream = b->stream;
    return L;
}

// The stages of one step of every problem, stage after stage, each one batched launch
// per class, all on the batch stream; timed: an event before every launch group (stage,
// class) and one at the end (outside any graph).
static void batch_harvest(adg_batch *b, int g) {
    const size_t nl = BSTAGE_COUNT * b->cls.size();
    for (size_t i = 0; i < nl; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev[g][i], b->ev[g][i + 1]) == hipSuccess) b->prof_ms[i] += ms;
    }
    b->prof_n += 1;
    b->ev_pending[g] = false;
}

static int batch_enqueue(adg_batch *b, int g, bool timed) {
    const int nc = (int)b->cls.size();
    if (timed && b->ev_pending[g]) {
        // this parity's events of the previous step: add them up before recording again
        HIPCHK(hipEventSynchronize(b->ev[g][BSTAGE_COUNT * nc]));
        batch_harvest(b, g);
    }
    for (int st = 0; st < BSTAGE_COUNT; st++) {
        const bool lim_stage = st == BSTAGE_BOUNDS || st == BSTAGE_COMPACT || st == BSTAGE_SUBCELL ||
                               st == BSTAGE_FLUXCORR;
        for (int c = 0; c < nc; c++) {
            if (timed) HIPCHK(hipEventRecord(b->ev[g][st * nc + c], b->stream));
            if (lim_stage && !b->limiter) continue;
            const BatchClass &K = b->cls[c];
            launch_batched(K.dim, K.N, st, batch_launch(b, K, g));
        }
    }
    if (timed) {
        HIPCHK(hipEventRecord(b->ev[g][BSTAGE_COUNT * nc], b->stream));
        b->ev_pending[g] = true;
    }
    HIPCHK(hipGetLastError());
    return ADG_OK;
}

static int batch_capture(adg_batch *b) {
    // entries of both parities from the problems' current buffers
    for (const auto &K : b->cls) {
        for (int g = 0; g < 2; g++) {
            std::vector<BatchEntry> ents;
            for (int m : K.members) ents.push_back(batch_entry(b->ps[m], g, b->cfl, b->precision));
            HIPCHK(hipMemcpyAsync(b->ws + K.off_ents[g], ents.data(), sizeof(BatchEntry) * ents.size(),
                                  hipMemcpyHostToDevice, b->stream));
        }
        for (int t = 0; t < 6; t++)
            if (!K.tiles[t].empty())
                HIPCHK(hipMemcpyAsync(b->ws + K.off_tiles[t], K.tiles[t].data(), sizeof(BTile) * K.tiles[t].size(),
                                      hipMemcpyHostToDevice, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int g = 0; g < 2; g++) {
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const int rc = batch_enqueue(b, g, false);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &gr);
        if (rc != ADG_OK) return rc;
        if (e != hipSuccess) return fail(ADG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph[g] = gr;
        HIPCHK(hipGraphInstantiate(&b->exec[g], gr, nullptr, nullptr, 0));
    }
    b->parity = 0;
    b->captured = true;
    return ADG_OK;
}

static void batch_drop_graphs(adg_batch *b) {
    for (int g = 0; g < 2; g++) {
        if (b->exec[g]) (void)hipGraphExecDestroy(b->exec[g]);
        if (b->graph[g]) (void)hipGraphDestroy(b->graph[g]);
        b->exec[g] = nullptr;
        b->graph[g] = nullptr;
    }
    b->captured = false;
}

extern "C" {

int adg_batch_create(adg_problem *const *ps, int count, adg_batch **out) {
    if (!ps || count <= 0 || !out) return fail(ADG_EINVAL, "bad argument");
    *out = nullptr;
    for (int i = 0; i < count; i++) {
        adg_problem *pb = ps[i];
        if (!pb || !pb->has_state) return fail(ADG_ESTATE, "problem %d has no state", i);
        if (pb->batch) return fail(ADG_ESTATE, "problem %d already belongs to a batch", i);
        for (int j = 0; j < i; j++)
            if (ps[j] == pb) return fail(ADG_EINVAL, "problem listed twice");
        const adg_params &a = ps[0]->prm, &c = pb->prm;
        if (c.precision != a.precision || c.limiter != a.limiter || c.mood != a.mood)
            return fail(ADG_EINVAL, "problem %d: the problems of a batch share precision, limiter and MOOD layer", i);
        if (big_slot_doubles(pb->P.dim, pb->P.N) > 0)
            return fail(ADG_EINVAL, "problem %d: 3D problems of degree %d are stepped one by one, not in a batch", i,
                        pb->P.N);
    }
    adg_batch *b = new (std::nothrow) adg_batch();
    if (!b) return fail(ADG_ENOMEM, "host allocation failed");
    b->ps.assign(ps, ps + count);
    b->precision = ps[0]->prm.precision;
    b->limiter = ps[0]->prm.limiter;
    b->mood = ps[0]->prm.mood;
    for (int i = 0; i < count; i++) {
        b->saved.push_back(ps[i]->stream);
        int k = -1;
        for (size_t j = 0; j < b->cls.size(); j++)
            if (b->cls[j].dim == ps[i]->P.dim && b->cls[j].N == ps[i]->P.N) k = (int)j;
        if (k < 0) {
            b->cls.emplace_back();
            b->cls.back().dim = ps[i]->P.dim;
            b->cls.back().N = ps[i]->P.N;
            k = (int)b->cls.size() - 1;
        }
        b->cls[k].members.push_back(i);
    }
    for (int g = 0; g < 2; g++) {
        b->ev[g].assign(BSTAGE_COUNT * b->cls.size() + 1, nullptr);
        for (auto &e : b->ev[g])
            if (hipEventCreate(&e) != hipSuccess) {
                adg_batch_destroy(b);
                return fail(ADG_EDEVICE, "hipEventCreate failed");
            }
    }
    b->prof_ms.assign(BSTAGE_COUNT * b->cls.size(), 0.0);
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        adg_batch_destroy(b);
        return fail(ADG_EDEVICE, "hipStreamCreate failed");
    }
    batch_plan(b);
    for (auto *pb : b->ps) pb->batch = b;
    *out = b;
    return ADG_OK;
}

size_t adg_batch_workspace_bytes(const adg_batch *b) { return b ? b->ws_bytes : 0; }

int adg_batch_bind(adg_batch *b, void *dev_workspace, size_t bytes, void *hip_stream) {
    if (!b || !dev_workspace) return fail(ADG_EINVAL, "null argument");
    if (((uintptr_t)dev_workspace) & 255) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < b->ws_bytes) return fail(ADG_ENOMEM, "batch workspace %zu bytes, %zu needed", bytes, b->ws_bytes);
    batch_drop_graphs(b);
    b->ws = (char *)dev_workspace;
    b->user = (hipStream_t)hip_stream;
    b->bound = true;
    return ADG_OK;
}

int adg_batch_step_cfl(adg_batch *b, double cfl, int nsteps) {
    if (!b || !(cfl > 0) || nsteps < 0) return fail(ADG_EINVAL, "bad argument");
    if (!b->bound) return fail(ADG_ESTATE, "adg_batch_bind first");
    // make the caller's and the problems' pending work visible to the batch stream
    HIPCHK(hipStreamSynchronize(b->user));
    for (size_t i = 0; i < b->ps.size(); i++) HIPCHK(hipStreamSynchronize(b->saved[i]));
    int done = 0;
    if (!b->captured || b->cfl != cfl) {
        batch_drop_graphs(b);
        b->cfl = cfl;
        // one ordinary step per problem (initialises the old-time bounds), then capture
        if (nsteps > 0) {
            for (size_t i = 0; i < b->ps.size(); i++) {
                adg_problem *pb = b->ps[i];
                pb->stream = b->stream;
                pb->batch_driving = true;
                int rc = adg_step_cfl(pb, cfl);
                pb->batch_driving = false;
                pb->stream = b->saved[i];
                if (rc != ADG_OK && rc != ADG_ENONPHYSICAL) return rc;
            }
            done = 1;
        }
        HIPCHK(hipStreamSynchronize(b->stream));
        for (auto *pb : b->ps)
            if (!pb->bounds_valid && b->limiter)
                return fail(ADG_ESTATE, "batch capture needs one step taken (nsteps >= 1)");
        int rc = batch_capture(b);
        if (rc != ADG_OK) return rc;
    }
    const bool timed = b->prof_mask != 0;
    for (int s = done; s < nsteps; s++) {
        const int g = b->parity;
        if (timed) {
            // the same launches as the graph, enqueued directly with an event at every stage
            // boundary (events recorded inside a graph give no elapsed times here)
            int rc = batch_enqueue(b, g, true);
            if (rc != ADG_OK) return rc;
        } else {
            HIPCHK(hipGraphLaunch(b->exec[g], b->stream));
        }
        for (auto *pb : b->ps) host_advance(pb);
        b->parity ^= 1;
    }
    if (timed && nsteps > done) {
        HIPCHK(hipStreamSynchronize(b->stream));
        for (int g = 0; g < 2; g++)
            if (b->ev_pending[g]) batch_harvest(b, g);
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    // the replays do not copy the counters to the host: read every problem's pool
    // overflow flag (sticky) and its count of non-physical subcell results now
    for (auto *pb : b->ps) HIPCHK(hipMemcpyAsync(pb->pinned, pb->B.counts, 16, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    int news = ADG_OK;
    for (size_t i = 0; i < b->ps.size(); i++) {
        adg_problem *pb = b->ps[i];
        if (pb->pinned[3])
            return fail(ADG_ECAPACITY, "problem %d: troubled cells exceeded the pool capacity %lld", (int)i,
                        (long long)pb->cap);
        if (nonphysical_news(pb) != ADG_OK) news = ADG_ENONPHYSICAL;
    }
    if (news != ADG_OK) return fail(ADG_ENONPHYSICAL, "subcell results failed positivity in the batch");
    return ADG_OK;
}

int adg_batch_profile(adg_batch *b, int enable) {
    if (!b) return fail(ADG_EINVAL, "null argument");
    b->prof_mask = enable ? 1u : 0u;
    b->ev_pending[0] = b->ev_pending[1] = false;
    std::fill(b->prof_ms.begin(), b->prof_ms.end(), 0.0);
    b->prof_n = 0;
    return ADG_OK;
}

int adg_batch_classes(const adg_batch *b, int *dims, int *Ns, int max_classes) {
    if (!b) return fail(ADG_EINVAL, "null argument");
    const int nc = (int)b->cls.size();
    for (int c = 0; c < nc && c < max_classes; c++) {
        if (dims) dims[c] = b->cls[c].dim;
        if (Ns) Ns[c] = b->cls[c].N;
    }
    return nc;
}

int adg_batch_profile_read(adg_batch *b, double *ms, int64_t *steps) {
    if (!b || !ms || !steps) return fail(ADG_EINVAL, "null argument");
    std::copy(b->prof_ms.begin(), b->prof_ms.end(), ms);
    *steps = b->prof_n;
    return ADG_OK;
}

int adg_batch_dt(adg_batch *b, double *dts) {
    if (!b || !dts) return fail(ADG_EINVAL, "bad argument");
    for (size_t i = 0; i < b->ps.size(); i++) {
        double s[1];
        HIPCHK(hipMemcpy(s, b->ps[i]->B.scal, sizeof s, hipMemcpyDeviceToHost));
        dts[i] = s[0];
    }
    return ADG_OK;
}

int adg_batch_destroy(adg_batch *b) {
    if (!b) return ADG_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    if (b->stream) (void)hipStreamDestroy(b->stream);

    for (int g = 0; g < 2; g++)
        for (auto e : b->ev[g])
            if (e) (void)hipEventDestroy(e);
    for (size_t i = 0; i < b->ps.size(); i++) {
        b->ps[i]->stream = b->saved[i];
        if (b->ps[i]->batch == b) b->ps[i]->batch = nullptr;
    }
    delete b;
    return ADG_OK;
}

int adg_debug_poison(adg_problem *pb, int64_t cell, int var, double value) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    if (cell < 0 || cell >= pb->P.ncell || var < 0 || var >= pb->P.nv)
        return fail(ADG_EINVAL, "poison: cell %lld or variable %d out of range", (long long)cell, var);
    // armed flag, cell, variable, value: read by the next corrector, cleared at the end of that step
    const double rec[4] = {1.0, (double)cell, (double)var, value};
    HIPCHK(hipMemcpyAsync(pb->B.scal + 4, rec, sizeof rec, hipMemcpyHostToDevice, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    return ADG_OK;
}

// ------------------------------------------------- time step without a workspace
// The per-block partial maxima of the wave-speed reduction (at most ADG_STATIC_PARTIALS
// blocks) and the reduction's scalars, for adg_cfl_dt_static.  Each device holds its own
// copy until the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host it is only a stand-in for the device symbol): it uses the device address that
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) double scratch[ADG_STATIC_PARTIALS + 8];
static std::mutex g_scratch_mu;
static double *g_scratch_dev[64];   // per device ordinal: device address of `scratch`

static int scratch_for_current_device(double **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(ADG_EDEVICE, "device ordinal %d beyond 63", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ADG_EDEVICE, "hipGetSymbolAddress gave no address for the static scratch");
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return ADG_OK;
}

int adg_cfl_dt_static(const double *dev_u, int dim, int N, int64_t ncell, double gamma, double hmin, double cfl,
                      double *dev_dt, void *hip_stream) {
    if (!dev_u || !dev_dt) return fail(ADG_EINVAL, "null pointer");
    if (!supported(dim, N)) return fail(ADG_EINVAL, "dim %d, N %d not supported", dim, N);
    if (ncell < 1 || ncell > ADG_STATIC_MAX_CELLS)
        return fail(ADG_EINVAL, "ncell %lld outside 1..%lld", (long long)ncell, (long long)ADG_STATIC_MAX_CELLS);
    if (!(gamma > 1.0) || !(hmin > 0.0) || !(cfl > 0.0)) return fail(ADG_EINVAL, "gamma, hmin and cfl must be > 0 (gamma > 1)");
    double *ptr = nullptr;
    const int rc = scratch_for_current_device(&ptr);
    if (rc != ADG_OK) return rc;
    StepCtx C;
    std::memset((void *)&C, 0, sizeof C);
    C.P.dim = dim;
    C.P.N = N;
    C.P.n = N + 1;
    C.P.nv = dim + 2;
    C.P.ncell = ncell;
    C.P.gamma = gamma;
    C.B.lam_part = ptr;                          // partial maxima: ptr[0 .. ADG_STATIC_PARTIALS)
    C.B.scal = ptr + ADG_STATIC_PARTIALS;        // [0] dt, [2] largest signal speed
    C.stream = (hipStream_t)hip_stream;
    const int64_t nn = ipow64(N + 1, dim);
    C.lam_blocks = (int)std::min<int64_t>(ADG_STATIC_PARTIALS, std::max<int64_t>(1, (ncell * nn + 255) / 256));
    launch_lambda(C, dev_u, cfl * hmin / (dim * (2.0 * N + 1.0)));
    launch_copy_scalar(C.B.scal, dev_dt, C.stream);
    HIPCHK(hipGetLastError());
    return ADG_OK;
}

int adg_debug_force_troubled(adg_problem *pb, const uint8_t *mask) {
    if (!pb) return fail(ADG_EINVAL, "null argument");
    if (!pb->bound) return fail(ADG_ESTATE, "not bound");
    if (mask) HIPCHK(hipMemcpyAsync(pb->B.force, mask, pb->P.ncell, hipMemcpyHostToDevice, pb->stream));
    else HIPCHK(hipMemsetAsync(pb->B.force, 0, pb->P.ncell, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    return ADG_OK;
}

}  // extern "C"
