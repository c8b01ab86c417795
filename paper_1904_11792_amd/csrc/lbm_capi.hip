// Host runtime of liblbm: the C ABI declared in include/liblbm.h.
//
// A context borrows one caller-owned device workspace, carved as
//   [lattice 0][lattice 1][diag partials][slice maxima][latest record][ring]
// and orders all work on the caller's HIP stream.  Nothing here allocates
// device memory on the step path.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <cstdint>
#include <cmath>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/liblbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage) {
    switch (storage) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        default: return 2;
    }
}

bool is_mass_rest(int st) { return st == LBM_F16M || st == LBM_BF16M; }

int validate_params(const lbm_params *p) {
    if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_ERR_INVALID_ARG, "grid extents must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
    // Offsets within a z plane (19 nx ny populations, 20 slots per node with
    // an FP32 rest population) and node indices are 32-bit.
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
    if (int64_t(Q + 1) * p->nx * (int64_t(p->ny) + 31) > int64_t(0x7fffffff))
        return fail(LBM_ERR_INVALID_ARG, "a %d x %d plane holds more than 2^31 - 1 populations", p->nx, p->ny);
    if (n > int64_t(0x7fffffff))
        return fail(LBM_ERR_INVALID_ARG, "grid of %lld nodes exceeds 2^31 - 1 nodes", (long long)n);
    // the step kernels address within a plane with 32-bit byte offsets
    if (p->storage >= LBM_F64 && p->storage <= LBM_BF16M &&
        int64_t(Q + 1) * p->nx * (int64_t(p->ny) + 31) * int64_t(elem_bytes(p->storage)) > int64_t(0xffffffff))
        return fail(LBM_ERR_INVALID_ARG, "a %d x %d plane of this storage kind exceeds 4 GiB", p->nx, p->ny);
    if (!(p->tau > 0.5) || !isfinite(p->tau))
        return fail(LBM_ERR_INVALID_ARG, "tau must be finite and > 0.5 (got %g)", p->tau);
    if (!isfinite(p->G)) return fail(LBM_ERR_INVALID_ARG, "G must be finite");
    if (p->psi != LBM_PSI_EXP) return fail(LBM_ERR_UNSUPPORTED, "psi form %d is not provided", p->psi);
    if (!(p->rho0 > 0.0) || !isfinite(p->rho0))
        return fail(LBM_ERR_INVALID_ARG, "rho0 must be finite and > 0");
    if (p->storage < LBM_F64 || p->storage > LBM_BF16M)
        return fail(LBM_ERR_INVALID_ARG, "unknown storage kind %d", p->storage);
    if (!isfinite(p->rho_ref)) return fail(LBM_ERR_INVALID_ARG, "rho_ref must be finite");
    return LBM_OK;
}

struct Layout {
    int64_t S;       // population stride (elements)
    int R, P;        // record and plane strides (elements)
    int rec_shift;   // rows per record = 2^rec_shift
    size_t lat_bytes, off_lat1, off_part, off_slices, off_latest, off_ring, off_counter, total;
    int nparts, nslices;
};

// Rows per record: the smallest power of two k (and at most ny / 2) whose
// population segment, k nx elements, holds at least the target: 32 KiB with
// k <= 32 when nx is a power of two from 64 to 1024 and the grid (2^22 nodes
// or more) lives in HBM, 2 KiB with k <= 8 otherwise (on cache-resident grids
// the long records measured up to 6% slower, 64 x 64 x 144 FP64).  Measured on MI355X (default launches, HIP events, against the
// 2 KiB rule): power-of-two widths 64-512 3-5.5% faster in FP32 and FP64
// (256 x 256 x 1024 FP32 1.909 -> 1.808 ms; k = 64 and beyond slower again),
// about 1% in FP16S; other widths (24-480) equal or up to 2.6% slower with
// the larger records, and fastest with segments of about 2 KiB (rows of
// 24-112 nodes 6-21% faster at k = 8 than at k = 1).
int record_shift(int nx, int ny, int nz, int storage) {
    const bool in_hbm = int64_t(nx) * ny * nz >= (int64_t(1) << 22);
    const bool pow2 = in_hbm && nx >= 64 && nx <= 1024 && (nx & (nx - 1)) == 0;
    const size_t target = pow2 ? 32768 : 2048;
    const int smax = pow2 ? 5 : 3;
    int s = 0;
    while (s < smax && size_t(nx) * elem_bytes(storage) * (size_t(1) << s) < target && (2 << s) <= ny) ++s;
    return s;
}

// Rows padded to whole records.
int64_t padded_rows(int ny, int rec_shift) {
    const int64_t k = int64_t(1) << rec_shift;
    return (ny + k - 1) / k * k;
}

Layout layout_of(const lbm_params *p) {
    Layout L;
    // Records of k rows, [z][y / k][a][y % k][x]: the 19 population segments
    // of k grid rows are contiguous (population stride k nx, record stride
    // 19 k nx, plane stride 19 nx ny' with ny' = ny rounded up to records).
    // (kMassRest kinds: 20 slots of 16 bits per node, the FP32 rest
    // population taking the first two)
    L.rec_shift = record_shift(p->nx, p->ny, p->nz, p->storage);
    const int k = 1 << L.rec_shift;
    const int64_t nyp = padded_rows(p->ny, L.rec_shift);
    const int slots = storage_slots(is_mass_rest(p->storage));
    L.S = int64_t(k) * p->nx;
    L.R = slots * k * p->nx;
    L.P = int(int64_t(slots) * p->nx * nyp);
    const int64_t cells = int64_t(slots) * p->nx * nyp * p->nz;
    L.lat_bytes = align_up(size_t(cells) * elem_bytes(p->storage), 256);
    L.off_lat1 = L.lat_bytes;
    L.nparts = diag_blocks(p->nx, p->ny, p->nz);
    L.nslices = p->nx > p->ny ? (p->nx > p->nz ? p->nx : p->nz) : (p->ny > p->nz ? p->ny : p->nz);
    L.off_part = 2 * L.lat_bytes;
    L.off_slices = L.off_part + align_up(sizeof(DiagPartial) * L.nparts, 256);
    L.off_latest = L.off_slices + align_up(sizeof(unsigned long long) * L.nslices, 256);
    L.off_ring = L.off_latest + align_up(sizeof(DiagRecord), 256);
    L.off_counter = L.off_ring + align_up(sizeof(DiagRecord) * LBM_DIAG_RING, 256);
    L.total = L.off_counter + 256;
    return L;
}

bool is_shifted(int st) { return st == LBM_F16S || st == LBM_BF16S || st == LBM_F16M || st == LBM_BF16M; }

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// ---- tiny JSON cache of tuned launch shapes: {"key": [tx, ty, zchunk], ...}
std::string tune_key(const lbm_params *p) {
    char buf[160];
    snprintf(buf, sizeof(buf), "%s:%d:%dx%dx%d", arch_name().c_str(), p->storage, p->nx, p->ny, p->nz);
    return buf;
}

bool cache_lookup(const std::string &key, lbm_launch *out) {
    const char *path = getenv("LBM_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    fclose(f);
    const std::string pat = "\"" + key + "\"";
    const size_t at = s.find(pat);
    if (at == std::string::npos) return false;
    int tx, ty, zc;
    if (sscanf(s.c_str() + at + pat.size(), " : [%d , %d , %d]", &tx, &ty, &zc) != 3) return false;
    out->tile_x = tx;
    out->tile_y = ty;
    out->zchunk = zc;
    return true;
}

void cache_store(const std::string &key, const lbm_launch &l) {
    const char *path = getenv("LBM_TUNE_CACHE");
    if (!path || !*path) return;
    std::vector<std::pair<std::string, lbm_launch>> entries;
    if (FILE *f = fopen(path, "r")) {
        std::string s;
        char buf[4096];
        size_t k;
        while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
        fclose(f);
        size_t pos = 0;
        while ((pos = s.find('"', pos)) != std::string::npos) {
            const size_t end = s.find('"', pos + 1);
            if (end == std::string::npos) break;
            std::string k2 = s.substr(pos + 1, end - pos - 1);
            lbm_launch e;
            if (sscanf(s.c_str() + end + 1, " : [%d , %d , %d]", &e.tile_x, &e.tile_y, &e.zchunk) == 3 &&
                k2 != key)
                entries.emplace_back(k2, e);
            pos = end + 1;
        }
    }
    entries.emplace_back(key, l);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i)
        fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", entries[i].first.c_str(), entries[i].second.tile_x,
                entries[i].second.tile_y, entries[i].second.zchunk, i + 1 < entries.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

// Tile width/height of a launch on an nx x ny cross-section (tile_x = 0
// selects the run-time shaped tile).
void tile_dims(const lbm_launch &l, int nx, int ny, int *tw, int *th) {
    if (l.tile_x == 0)
        dynamic_tile(l.tile_y, nx, ny, tw, th);
    else {
        *tw = l.tile_x;
        *th = l.tile_y;
    }
}

// Default launch shape: the run-time shaped tile, which spans whole rows up to
// 256 nodes (whole rows of the row-interleaved layout stream best), and about
// one workgroup per compute unit (256) by choosing the z chunk.
lbm_launch default_launch(const lbm_params *p) {
    lbm_launch l;
    l.tile_x = 0;  // full-row tile shaped at run time
    // 1024 threads for wide grids; FP64 keeps 512 (its kernel needs more than
    // the 128 VGPRs a 1024-thread workgroup allows)
    l.tile_y = (p->nx >= 128 && p->storage != LBM_F64) ? 1024 : 512;
    int tw, th;
    tile_dims(l, p->nx, p->ny, &tw, &th);
    const int64_t tiles = int64_t((p->nx + tw - 1) / tw) * ((p->ny + th - 1) / th);
    // A z chunk re-gathers two extra planes for psi.  Small grids (under 2^22
    // nodes) live in the caches, where more workgroups pay more than the extra
    // gathers cost: about 256 workgroups with chunks down to one plane
    // (32x32x64 on MI355X: 1.7x (FP32) and 1.9x (FP64) faster at chunks of 1
    // than of 4).
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
    if (n < (int64_t(1) << 22)) {
        const int64_t chunks = (256 + tiles - 1) / tiles;
        const int64_t zc = (p->nz + chunks - 1) / chunks;
        l.zchunk = int(zc < 1 ? 1 : zc);
        return l;
    }
    // Grids in HBM: chunks of at least 4 planes, and a launch that runs in
    // rounds of `slots` workgroups (those resident at once).  Cost model:
    // rounds x (z chunk + kRoundPlanes), where kRoundPlanes charges each
    // round's start-up, boundary re-gathers and tail in plane times (about 18,
    // measured on MI355X: 256x256x1024 FP32 with 512 workgroups of 128 planes
    // takes 1.067x the time of 256 of 256).  A count of workgroups just above
    // a multiple of the slots costs a whole extra round, which the model
    // avoids.
    constexpr int64_t kRoundPlanes = 18, kMinChunk = 4;
    int64_t slots = launch_slots(find_tile(l.tile_x, l.tile_y), p->storage);
    if (slots <= 0) slots = 256;
    int64_t best_zc = p->nz, best_cost = INT64_MAX;
    for (int64_t k = 1; k <= p->nz && k <= 65536; ++k) {
        const int64_t zc = (p->nz + k - 1) / k;
        if (zc < kMinChunk) break;
        if (k > 1 && zc == (p->nz + k - 2) / (k - 1)) continue;  // same chunk as k - 1
        const int64_t wgs = tiles * ((p->nz + zc - 1) / zc);
        const int64_t cost = (wgs + slots - 1) / slots * (zc + kRoundPlanes);
        if (cost < best_cost) {
            best_cost = cost;
            best_zc = zc;
        }
    }
    if (best_zc > p->nz) best_zc = p->nz;
    l.zchunk = int(best_zc);
    return l;
}

int check_launch(const lbm_launch *l, int storage) {
    if (!l) return fail(LBM_ERR_INVALID_ARG, "launch is NULL");
    const int ti = find_tile(l->tile_x, l->tile_y);
    if (ti < 0) return fail(LBM_ERR_UNSUPPORTED, "tile %dx%d is not compiled in", l->tile_x, l->tile_y);
    if (!tile_has_storage(ti, storage))
        return fail(LBM_ERR_UNSUPPORTED, "tile %dx%d is not compiled for storage kind %d (run-time tiles only)",
                    l->tile_x, l->tile_y, storage);
    if (l->zchunk < 1) return fail(LBM_ERR_INVALID_ARG, "zchunk must be >= 1");
    return LBM_OK;
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Layout lay;
    void *lat[2];
    int cur;
    int axis;
    int64_t step;
    bool initialized;
    bool poisoned;
    lbm_launch launch;
    int tile_index;
    DiagPartial *partials;
    unsigned long long *slices;
    DiagRecord *latest;
    DiagRecord *ring;
    int64_t ring_written, ring_read;
    int graph_chunk;
    hipGraphExec_t gexec;
    lbm_launch graph_launch;
    MrtParams mrt;  // collision operator (mrt.on = 0: BGK)
    // Device step counter read by the step kernels (the key of the
    // stochastic rounding): a launch's step is *counter + step_add.  dstep is
    // the value the counter holds when the next enqueued launch runs.
    uint32_t *counter;
    uint32_t dstep;
};

namespace {

int device_fail(lbm_ctx *c, hipError_t e, const char *what) {
    if (c) c->poisoned = true;
    return fail(LBM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_ctx(const lbm_ctx *c) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "context is NULL");
    if (c->poisoned) return fail(LBM_ERR_STATE, "context is poisoned by an earlier device error");
    return LBM_OK;
}

LatticeRef lattice_ref(const lbm_ctx *c, int which) {
    LatticeRef L;
    L.lat = c->lat[which];
    L.nx = c->p.nx;
    L.ny = c->p.ny;
    L.nz = c->p.nz;
    L.storage = c->p.storage;
    L.pop_stride = c->lay.S;
    L.row_stride = c->lay.R;
    L.plane_stride = c->lay.P;
    L.rec_shift = c->lay.rec_shift;
    L.rho_ref = is_shifted(c->p.storage) ? c->p.rho_ref : 0.0;
    L.frozen = nullptr;
    L.pair[0] = L.pair[1] = nullptr;
    return L;
}

StepArgs step_args(const lbm_ctx *c, const lbm_launch &l, int src) {
    StepArgs A;
    A.src = c->lat[src];
    A.dst = c->lat[src ^ 1];
    A.nx = c->p.nx;
    A.ny = c->p.ny;
    A.nz = c->p.nz;
    tile_dims(l, c->p.nx, c->p.ny, &A.tile_w, &A.tile_h);
    A.tiles_x = (c->p.nx + A.tile_w - 1) / A.tile_w;
    A.tiles_y = (c->p.ny + A.tile_h - 1) / A.tile_h;
    A.zchunk = l.zchunk < c->p.nz ? l.zchunk : c->p.nz;
    A.nchunks = (c->p.nz + A.zchunk - 1) / A.zchunk;
    A.pop_stride = c->lay.S;
    A.row_stride = c->lay.R;
    A.plane_stride = c->lay.P;
    A.rec_shift = c->lay.rec_shift;
    A.tau = c->p.tau;
    A.G = c->p.G;
    A.rho0 = c->p.rho0;
    A.rho_ref = is_shifted(c->p.storage) ? c->p.rho_ref : 0.0;
    A.mrt = c->mrt;
    A.step_base = c->counter;
    A.step_add = uint32_t(c->step) - c->dstep;
    return A;
}

hipError_t plain_steps(lbm_ctx *c, int64_t n) {
    const int ti = c->tile_index;
    for (int64_t s = 0; s < n; ++s) {
        const StepArgs A = step_args(c, c->launch, c->cur);
        hipError_t e = launch_step(ti, c->p.storage, A, c->stream);
        if (e != hipSuccess) return e;
        c->cur ^= 1;
        c->step += 1;
    }
    return hipSuccess;
}

void release_graph(lbm_ctx *c) {
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
}

// Capture graph_chunk steps starting from lattice 0, the s-th at step
// *counter + s, then the counter's advance by graph_chunk.
hipError_t build_graph(lbm_ctx *c) {
    release_graph(c);
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int s = 0; s < c->graph_chunk; ++s) {
        StepArgs A = step_args(c, c->launch, s & 1);
        A.step_add = uint32_t(s);
        e = launch_step(c->tile_index, c->p.storage, A, c->stream);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = launch_counter(c->counter, uint32_t(c->graph_chunk), true, c->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    c->graph_launch = c->launch;
    return e;
}

int get_fields_impl(lbm_ctx *c, const LatticeRef &L, const lbm_params &p, hipStream_t stream,
                    uint32_t mask, double *rho, double *u, double *force, double *pop, int32_t on_device) {
    const int64_t n = int64_t(p.nx) * p.ny * p.nz;
    if (mask & ~uint32_t(LBM_FIELD_RHO | LBM_FIELD_U | LBM_FIELD_FORCE | LBM_FIELD_POP))
        return fail(LBM_ERR_INVALID_ARG, "unknown field bits in mask 0x%x", mask);
    if (((mask & LBM_FIELD_RHO) && !rho) || ((mask & LBM_FIELD_U) && !u) ||
        ((mask & LBM_FIELD_FORCE) && !force) || ((mask & LBM_FIELD_POP) && !pop))
        return fail(LBM_ERR_INVALID_ARG, "a requested field has a NULL pointer");
    const bool need_rho = mask & (LBM_FIELD_RHO | LBM_FIELD_U | LBM_FIELD_FORCE);
    // device destinations (either the caller's or temporaries)
    double *d_rho = nullptr, *d_u = nullptr, *d_f = nullptr, *d_pop = nullptr;
    std::vector<void *> temps;
    auto temp = [&](size_t count, double **out) -> hipError_t {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, count * sizeof(double));
        if (e == hipSuccess) temps.push_back(q);
        *out = static_cast<double *>(q);
        return e;
    };
    hipError_t e = hipSuccess;
    if (on_device) {
        d_rho = (mask & LBM_FIELD_RHO) ? rho : nullptr;
        d_u = (mask & LBM_FIELD_U) ? u : nullptr;
        d_f = (mask & LBM_FIELD_FORCE) ? force : nullptr;
        d_pop = (mask & LBM_FIELD_POP) ? pop : nullptr;
        if (need_rho && !d_rho) e = temp(n, &d_rho);
    } else {
        if (need_rho && e == hipSuccess) e = temp(n, &d_rho);
        if ((mask & LBM_FIELD_U) && e == hipSuccess) e = temp(3 * n, &d_u);
        if ((mask & LBM_FIELD_FORCE) && e == hipSuccess) e = temp(3 * n, &d_f);
        if ((mask & LBM_FIELD_POP) && e == hipSuccess) e = temp(size_t(Q) * n, &d_pop);
    }
    if (e == hipSuccess && need_rho) e = launch_export_rho(L, d_rho, stream);
    if (e == hipSuccess && (d_u || d_f)) e = launch_export_force_u(L, d_rho, p.G, p.rho0, d_f, d_u, stream);
    if (e == hipSuccess && d_pop) e = launch_export_pop(L, d_pop, stream);
    if (e == hipSuccess && !on_device) {
        if (mask & LBM_FIELD_RHO) e = hipMemcpyAsync(rho, d_rho, n * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && (mask & LBM_FIELD_U))
            e = hipMemcpyAsync(u, d_u, 3 * n * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && (mask & LBM_FIELD_FORCE))
            e = hipMemcpyAsync(force, d_f, 3 * n * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && (mask & LBM_FIELD_POP))
            e = hipMemcpyAsync(pop, d_pop, size_t(Q) * n * sizeof(double), hipMemcpyDeviceToHost, stream);
    }
    if (!temps.empty() || !on_device) {
        hipError_t e2 = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = e2;
    }
    for (void *q : temps) (void)hipFree(q);
    if (e != hipSuccess) return device_fail(c, e, "lbm_get_fields");
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

const char *lbm_version(void) { return "liblbm 0.1 (gfx950)"; }

size_t lbm_workspace_bytes(const lbm_params *p) {
    if (validate_params(p) != LBM_OK) return 0;
    return layout_of(p).total;
}

int lbm_create(const lbm_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out) {
    int st = validate_params(p);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    if (!d_workspace) return fail(LBM_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
        return fail(LBM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const Layout lay = layout_of(p);
    if (ws_bytes < lay.total)
        return fail(LBM_ERR_BUFFER_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, lay.total);
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char *>(d_workspace);
    c->ws_bytes = ws_bytes;
    c->lay = lay;
    c->lat[0] = c->ws;
    c->lat[1] = c->ws + lay.off_lat1;
    c->partials = reinterpret_cast<DiagPartial *>(c->ws + lay.off_part);
    c->slices = reinterpret_cast<unsigned long long *>(c->ws + lay.off_slices);
    c->latest = reinterpret_cast<DiagRecord *>(c->ws + lay.off_latest);
    c->ring = reinterpret_cast<DiagRecord *>(c->ws + lay.off_ring);
    c->cur = 0;
    c->axis = 2;
    c->step = 0;
    c->initialized = false;
    c->poisoned = false;
    c->ring_written = c->ring_read = 0;
    c->graph_chunk = 0;
    c->gexec = nullptr;
    c->mrt = MrtParams{};
    c->counter = reinterpret_cast<uint32_t *>(c->ws + lay.off_counter);
    c->dstep = 0;
    lbm_launch l;
    if (!cache_lookup(tune_key(p), &l) || check_launch(&l, p->storage) != LBM_OK) l = default_launch(p);
    c->launch = l;
    c->tile_index = find_tile(l.tile_x, l.tile_y);
    hipError_t e = launch_fill_u64(c->slices, lay.nslices, 0ull, c->stream);
    if (e == hipSuccess) e = launch_counter(c->counter, 0u, false, c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(LBM_ERR_DEVICE, "lbm_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "context is NULL");
    // A captured graph may still be running on the stream: let it finish
    // before its executable is destroyed.
    if (c->gexec) (void)hipStreamSynchronize(c->stream);
    release_graph(c);
    delete c;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Equal-area (mechanical stability) construction of the Shan-Chen EOS,
// P = rho/3 + G psi^2/6 (Eq. 7), psi = rho0 (1 - exp(-rho/rho0)):
// P(rho_v) = P(rho_l) = p and the integral of (p - P) psi'/psi^2 from rho_v
// to rho_l vanishes.  Spinodals in closed form, branches and p by bisection,
// the integral by composite Simpson.  Used as the start of the flat-interface
// run.  Requires G < -4/rho0.
struct EqualArea {
    double G, rho0;
    double psi(double r) const { return -rho0 * expm1(-r / rho0); }
    double P(double r) const {
        const double s = psi(r);
        return r / 3.0 + G * s * s / 6.0;
    }
    template <typename F>
    static double bisect(F f, double a, double b) {  // f(a) < 0 < f(b)
        for (int i = 0; i < 200 && b - a > 1e-15 * (1.0 + fabs(b)); ++i) {
            const double m = 0.5 * (a + b);
            (f(m) < 0 ? a : b) = m;
        }
        return 0.5 * (a + b);
    }
    void solve(double *rl, double *rv) const {
        const double root = sqrt(1.0 + 4.0 / (G * rho0));
        const double s_lo = -rho0 * log(0.5 * (1.0 + root));
        const double s_hi = -rho0 * log(0.5 * (1.0 - root));
        auto branches = [&](double p, double *v, double *l) {
            *v = bisect([&](double r) { return P(r) - p; }, 0.0, s_lo);
            const double top = 3.0 * (p - G * rho0 * rho0 / 6.0) + 10.0;
            *l = bisect([&](double r) { return P(r) - p; }, s_hi, top);
        };
        // Simpson in u = ln(rho) (drho = rho du), where the integrand is smooth
        // down to small vapour densities.
        auto area = [&](double p) {
            double v, l;
            branches(p, &v, &l);
            const int N = 4000;
            const double u0 = log(v), h = (log(l) - u0) / N;
            double acc = 0.0;
            for (int i = 0; i <= N; ++i) {
                const double r = exp(u0 + i * h);
                const double s = psi(r);
                const double f = (p - P(r)) * exp(-r / rho0) / (s * s) * r;
                acc += f * (i == 0 || i == N ? 1.0 : (i & 1 ? 4.0 : 2.0));
            }
            return acc * h / 3.0;
        };
        double lo = P(s_hi) > 0.0 ? P(s_hi) : 0.0, hi = P(s_lo);
        const double eps = 1e-12 * (hi - lo);
        const double p = bisect(area, lo + eps, hi - eps);
        branches(p, rv, rl);
    }
};

}  // namespace

extern "C" {

int lbm_equal_area(double G, int32_t psi, double rho0, double *rho_l, double *rho_v) {
    if (!rho_l || !rho_v) return fail(LBM_ERR_INVALID_ARG, "output pointers are NULL");
    if (psi != LBM_PSI_EXP) return fail(LBM_ERR_UNSUPPORTED, "psi form %d is not provided", psi);
    if (!(rho0 > 0.0) || !isfinite(rho0)) return fail(LBM_ERR_INVALID_ARG, "rho0 must be > 0");
    if (!(G < -4.0 / rho0) || !isfinite(G))
        return fail(LBM_ERR_INVALID_ARG, "no liquid-vapour coexistence for G = %g (needs G < %g)", G, -4.0 / rho0);
    EqualArea{G, rho0}.solve(rho_l, rho_v);
    return LBM_OK;
}

}  // extern "C"

namespace {

int check_mrt(const lbm_mrt *m) {
    const double r[5] = {m->s_e, m->s_eps, m->s_q, m->s_pi, m->s_m};
    for (double v : r)
        if (!(v > 0.0 && v < 2.0)) return fail(LBM_ERR_INVALID_ARG, "MRT rates must lie in (0, 2)");
    if (!(m->s_j < 2.0) || !std::isfinite(m->s_j))
        return fail(LBM_ERR_INVALID_ARG, "s_j must be below 2 (or <= 0 for 1/tau)");
    return LBM_OK;
}

MrtParams mrt_params(const lbm_mrt *m) {
    MrtParams p{};
    if (m) {
        p.on = 1;
        p.s_e = m->s_e;
        p.s_eps = m->s_eps;
        p.s_q = m->s_q;
        p.s_pi = m->s_pi;
        p.s_m = m->s_m;
        p.s_j = m->s_j > 0.0 ? m->s_j : 0.0;
    }
    return p;
}

int check_coexistence_args(double G, double tau, int32_t psi, double rho0) {
    if (psi != LBM_PSI_EXP) return fail(LBM_ERR_UNSUPPORTED, "psi form %d is not provided", psi);
    if (!(tau > 0.5) || !isfinite(tau)) return fail(LBM_ERR_INVALID_ARG, "tau must be > 0.5");
    if (!(rho0 > 0.0) || !isfinite(rho0)) return fail(LBM_ERR_INVALID_ARG, "rho0 must be > 0");
    if (!(G < -4.0 / rho0) || !isfinite(G))
        return fail(LBM_ERR_INVALID_ARG, "no liquid-vapour coexistence for G = %g (needs G < %g)", G, -4.0 / rho0);
    return LBM_OK;
}

// Host side of one flat-interface run: the tau stages and the stopping rule.
// Relaxation stages for tau < 1: tau = 1, then lowered by 0.05 down to
// (excluding) the target, each until the chunk residual is below 1e-8 or 100
// chunks.  Then the target tau until the residual is below 1e-12, until it has
// grown 100-fold above its smallest value once that is below 1e-8, or for 200
// chunks; the densities of the chunk with the smallest residual are the result.
struct CoexRun {
    static constexpr int kStageChunks = 100, kFinalChunks = 200;
    double G, tau, rho0;
    MrtParams mrt;
    double start_l = 0, start_v = 0;
    std::vector<double> stages;
    size_t stage = 0;  // == stages.size(): at the requested tau
    int k = 0;         // chunks run in the current stage
    bool first = true, done = false, diverged = false;
    double best = INFINITY, bl = 0, bv = 0;

    CoexRun(double G_, double tau_, double rho0_, const MrtParams &m) : G(G_), tau(tau_), rho0(rho0_), mrt(m) {
        EqualArea{G, rho0}.solve(&start_l, &start_v);
        if (tau < 1.0)
            for (int i = 0;; ++i) {
                const double t = 1.0 - 0.05 * i;
                if (!(t > tau + 1e-12)) break;
                stages.push_back(t);
            }
    }
    double current_tau() const { return stage < stages.size() ? stages[stage] : tau; }
    // Takes the result of the chunk just run (out as in launch_coexistence_chunk).
    void take(const double *out) {
        first = false;
        ++k;
        if (stage < stages.size()) {
            if (out[3] != 0.0) {
                diverged = done = true;
            } else if (out[2] < 1e-8 || k >= kStageChunks) {
                ++stage;
                k = 0;
            }
            return;
        }
        if (out[3] != 0.0) {
            if (!(best < INFINITY)) diverged = true;
            done = true;
            return;
        }
        const double res = out[2];
        if (res < best) {
            best = res;
            bl = out[0];
            bv = out[1];
        }
        if (res < 1e-12 || (best < 1e-8 && res > 100.0 * best) || k >= kFinalChunks) done = true;
    }
};

constexpr int kCoexNodes = 128, kCoexChunk = 1000;

// Advances every run to its end, all unfinished runs in one launch per chunk
// (one workgroup each).  Synchronous.  Device buffers of the caller: d_state
// holds 19 * 128 doubles per run, d_out 4 doubles per run, d_cases one
// table entry per run.
hipError_t run_coexistence_in(std::vector<CoexRun> &runs, double *d_state, double *d_out, CoexCase *d_cases) {
    const int n = kCoexNodes, chunk = kCoexChunk;
    const size_t m = runs.size();
    hipError_t e = hipSuccess;
    std::vector<CoexCase> table;
    std::vector<size_t> idx;
    std::vector<double> outs(4 * m);
    while (e == hipSuccess) {
        table.clear();
        idx.clear();
        for (size_t j = 0; j < m; ++j) {
            const CoexRun &r = runs[j];
            if (r.done) continue;
            CoexCase c{};
            c.state = d_state + j * Q * n;
            c.out = d_out + 4 * j;
            c.G = r.G;
            c.tau = r.current_tau();
            c.rho0 = r.rho0;
            c.hi = r.start_l;
            c.lo = r.start_v;
            c.mrt = r.mrt;
            c.init = r.first ? 1 : 0;
            table.push_back(c);
            idx.push_back(j);
        }
        if (table.empty()) break;
        e = hipMemcpy(d_cases, table.data(), sizeof(CoexCase) * table.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_coexistence_chunk(d_cases, int(table.size()), n, chunk, nullptr);
        if (e == hipSuccess) e = hipMemcpy(outs.data(), d_out, sizeof(double) * 4 * m, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (size_t j : idx) runs[j].take(&outs[4 * j]);
    }
    return e;
}

// The same with temporaries allocated here and freed before returning.
hipError_t run_coexistence(std::vector<CoexRun> &runs) {
    const size_t m = runs.size();
    double *d_state = nullptr, *d_out = nullptr;
    CoexCase *d_cases = nullptr;
    hipError_t e = hipMalloc(&d_state, sizeof(double) * Q * kCoexNodes * m);
    if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(double) * 4 * m);
    if (e == hipSuccess) e = hipMalloc(&d_cases, sizeof(CoexCase) * m);
    if (e == hipSuccess) e = run_coexistence_in(runs, d_state, d_out, d_cases);
    if (d_cases) (void)hipFree(d_cases);
    if (d_out) (void)hipFree(d_out);
    if (d_state) (void)hipFree(d_state);
    return e;
}

int coexistence_impl(double G, double tau, const lbm_mrt *mrt_in, int32_t psi, double rho0, double *rho_l,
                     double *rho_v) {
    if (!rho_l || !rho_v) return fail(LBM_ERR_INVALID_ARG, "output pointers are NULL");
    if (mrt_in) {
        const int mst = check_mrt(mrt_in);
        if (mst != LBM_OK) return mst;
    }
    const int ast = check_coexistence_args(G, tau, psi, rho0);
    if (ast != LBM_OK) return ast;
    std::vector<CoexRun> runs{CoexRun(G, tau, rho0, mrt_params(mrt_in))};
    const hipError_t e = run_coexistence(runs);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, "lbm_coexistence: %s", hipGetErrorString(e));
    if (runs[0].diverged) return fail(LBM_ERR_DIVERGED, "flat interface diverged for G=%g tau=%g", G, tau);
    *rho_l = runs[0].bl;
    *rho_v = runs[0].bv;
    return LBM_OK;
}

// ---- the allocation-free variant of lbm_coexistence_many ----------------
//
// Its device memory is a file-scope array, one per GPU, held until the
// process ends: run states (19 x 128 doubles each), results (4 doubles each)
// and the case table, for at most LBM_NOALLOC_MAX_RUNS runs.  Host code
// reaches it only through the address hipGetSymbolAddress gives on each
// device (the array's name is a host-side stand-in, not a device address).
constexpr size_t kNoAllocStateBytes = sizeof(double) * Q * kCoexNodes * LBM_NOALLOC_MAX_RUNS;
constexpr size_t kNoAllocOutBytes = sizeof(double) * 4 * LBM_NOALLOC_MAX_RUNS;
constexpr size_t kNoAllocBytes = kNoAllocStateBytes + kNoAllocOutBytes + sizeof(CoexCase) * LBM_NOALLOC_MAX_RUNS;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
hipError_t noalloc_scratch(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_ptr[dev]);
    return hipSuccess;
}

int coexistence_many_impl(int32_t m, const double *G, const double *tau, const lbm_mrt *mrt, int32_t psi,
                          double rho0, double *rho_l, double *rho_v, int32_t *status, bool noalloc) {
    if (m < 1) return fail(LBM_ERR_INVALID_ARG, "m must be >= 1");
    if (!G || !tau || !rho_l || !rho_v || !status) return fail(LBM_ERR_INVALID_ARG, "an array pointer is NULL");
    if (mrt) {
        const int mst = check_mrt(mrt);
        if (mst != LBM_OK) return mst;
    }
    const MrtParams mp = mrt_params(mrt);
    std::vector<CoexRun> runs;
    runs.reserve(size_t(m));
    for (int32_t j = 0; j < m; ++j) {
        const int ast = check_coexistence_args(G[j], tau[j], psi, rho0);
        if (ast != LBM_OK) {
            const std::string msg = g_err;
            return fail(ast, "case %d: %s", j, msg.c_str());
        }
        runs.emplace_back(G[j], tau[j], rho0, mp);
    }
    hipError_t e = hipSuccess;
    if (noalloc) {
        char *base = nullptr;
        e = noalloc_scratch(&base);
        if (e == hipSuccess)
            e = run_coexistence_in(runs, reinterpret_cast<double *>(base),
                                   reinterpret_cast<double *>(base + kNoAllocStateBytes),
                                   reinterpret_cast<CoexCase *>(base + kNoAllocStateBytes + kNoAllocOutBytes));
    } else {
        e = run_coexistence(runs);
    }
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "%s: %s", noalloc ? "lbm_coexistence_many_noalloc" : "lbm_coexistence_many",
                    hipGetErrorString(e));
    int first_bad = -1, nbad = 0;
    for (int32_t j = 0; j < m; ++j) {
        const CoexRun &r = runs[size_t(j)];
        status[j] = r.diverged ? LBM_ERR_DIVERGED : LBM_OK;
        rho_l[j] = r.diverged ? NAN : r.bl;
        rho_v[j] = r.diverged ? NAN : r.bv;
        if (r.diverged && nbad++ == 0) first_bad = j;
    }
    if (nbad)
        return fail(LBM_ERR_DIVERGED, "%d of %d flat interfaces diverged (first: case %d, G=%g tau=%g)", nbad, m,
                    first_bad, G[first_bad], tau[first_bad]);
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_coexistence(double G, double tau, int32_t psi, double rho0, double *rho_l, double *rho_v) {
    return coexistence_impl(G, tau, nullptr, psi, rho0, rho_l, rho_v);
}

int lbm_coexistence_mrt(double G, double tau, const lbm_mrt *mrt, int32_t psi, double rho0, double *rho_l,
                        double *rho_v) {
    if (!mrt) return fail(LBM_ERR_INVALID_ARG, "mrt is NULL");
    return coexistence_impl(G, tau, mrt, psi, rho0, rho_l, rho_v);
}

int lbm_coexistence_many(int32_t m, const double *G, const double *tau, const lbm_mrt *mrt, int32_t psi,
                         double rho0, double *rho_l, double *rho_v, int32_t *status) {
    return coexistence_many_impl(m, G, tau, mrt, psi, rho0, rho_l, rho_v, status, false);
}

int lbm_coexistence_many_noalloc(int32_t m, const double *G, const double *tau, const lbm_mrt *mrt,
                                 int32_t psi, double rho0, double *rho_l, double *rho_v, int32_t *status) {
    if (m > LBM_NOALLOC_MAX_RUNS)
        return fail(LBM_ERR_INVALID_ARG, "lbm_coexistence_many_noalloc takes at most %d runs (got %d)",
                    int(LBM_NOALLOC_MAX_RUNS), m);
    return coexistence_many_impl(m, G, tau, mrt, psi, rho0, rho_l, rho_v, status, true);
}

int lbm_set_mrt(lbm_ctx *c, const lbm_mrt *mrt) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (mrt) {
        st = check_mrt(mrt);
        if (st != LBM_OK) return st;
    }
    if (mrt && is_mass_rest(c->p.storage))
        return fail(LBM_ERR_UNSUPPORTED, "the MRT collision is not provided for the FP32-rest storage kinds");
    c->mrt = mrt_params(mrt);
    if (c->mrt.on && !tile_has_mrt(c->tile_index)) {
        c->launch = default_launch(&c->p);  // a run-time tile, which has the MRT kernel
        c->tile_index = find_tile(c->launch.tile_x, c->launch.tile_y);
    }
    release_graph(c);
    return LBM_OK;
}

int lbm_init_ligament(lbm_ctx *c, const lbm_ligament *g) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!g) return fail(LBM_ERR_INVALID_ARG, "ligament spec is NULL");
    if (g->axis < 0 || g->axis > 2) return fail(LBM_ERR_INVALID_ARG, "axis must be 0, 1 or 2");
    if (!(g->R0 > 0) || !(g->wavelength > 0) || !(g->width > 0) || !(g->noise_amp >= 0) ||
        !isfinite(g->R0) || !isfinite(g->wavelength) || !isfinite(g->width) || !isfinite(g->amp_rel) ||
        !isfinite(g->c1) || !isfinite(g->c2) || !isfinite(g->noise_amp))
        return fail(LBM_ERR_INVALID_ARG, "ligament spec has a non-positive or non-finite field");
    LigamentArgs a;
    a.axis = g->axis;
    a.R0 = g->R0;
    a.amp_rel = g->amp_rel;
    a.wavelength = g->wavelength;
    a.c1 = g->c1;
    a.c2 = g->c2;
    a.width = g->width;
    a.rho_l = g->rho_l;
    a.rho_v = g->rho_v;
    a.noise_amp = g->noise_amp;
    a.seed = g->seed;
    if (!(a.rho_l > 0) || !(a.rho_v > 0)) {
        lbm_mrt m;
        if (c->mrt.on) {
            m.s_e = c->mrt.s_e;
            m.s_eps = c->mrt.s_eps;
            m.s_q = c->mrt.s_q;
            m.s_pi = c->mrt.s_pi;
            m.s_m = c->mrt.s_m;
            m.s_j = c->mrt.s_j;
        }
        st = coexistence_impl(c->p.G, c->p.tau, c->mrt.on ? &m : nullptr, c->p.psi, c->p.rho0, &a.rho_l,
                              &a.rho_v);
        if (st != LBM_OK) return st;
    }
    hipError_t e = launch_init_ligament(lattice_ref(c, 0), a, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "lbm_init_ligament");
    c->cur = 0;
    c->step = 0;
    c->initialized = true;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t nsteps) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (nsteps < 0) return fail(LBM_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    hipError_t e = hipSuccess;
    int64_t left = nsteps;
    if (c->graph_chunk > 0 && left >= c->graph_chunk) {
        if (c->cur == 1) {
            e = plain_steps(c, 1);
            left -= 1;
        }
        if (e == hipSuccess && (!c->gexec || memcmp(&c->graph_launch, &c->launch, sizeof(lbm_launch)) != 0))
            e = build_graph(c);
        if (e == hipSuccess && c->dstep != uint32_t(c->step)) {  // the graph counts from *counter
            e = launch_counter(c->counter, uint32_t(c->step), false, c->stream);
            c->dstep = uint32_t(c->step);
        }
        while (e == hipSuccess && left >= c->graph_chunk) {
            e = hipGraphLaunch(c->gexec, c->stream);
            c->step += c->graph_chunk;
            c->dstep += uint32_t(c->graph_chunk);
            left -= c->graph_chunk;
        }
    }
    if (e == hipSuccess) e = plain_steps(c, left);
    if (e != hipSuccess) return device_fail(c, e, "lbm_step");
    return LBM_OK;
}

int lbm_get_fields(lbm_ctx *c, uint32_t mask, double *rho, double *u, double *force, double *pop,
                   int32_t on_device) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    return get_fields_impl(c, lattice_ref(c, c->cur), c->p, c->stream, mask, rho, u, force, pop, on_device);
}

int lbm_set_populations(lbm_ctx *c, const double *pop, int32_t on_device) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!pop) return fail(LBM_ERR_INVALID_ARG, "pop is NULL");
    const int64_t n = int64_t(c->p.nx) * c->p.ny * c->p.nz;
    hipError_t e = hipSuccess;
    if (on_device) {
        e = launch_import(lattice_ref(c, c->cur), pop, c->stream);
    } else {
        double *d = nullptr;
        e = hipMalloc(&d, size_t(Q) * n * sizeof(double));
        if (e == hipSuccess) e = hipMemcpyAsync(d, pop, size_t(Q) * n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_import(lattice_ref(c, c->cur), d, c->stream);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = e2;
        if (d) (void)hipFree(d);
    }
    if (e != hipSuccess) return device_fail(c, e, "lbm_set_populations");
    c->initialized = true;
    return LBM_OK;
}

static void to_public(const DiagRecord &r, lbm_diag *out) {
    out->step = r.step;
    out->mass = r.mass;
    for (int d = 0; d < 3; ++d) out->mom[d] = r.mom[d];
    out->rho_min = r.rho_min;
    out->rho_max = r.rho_max;
    out->neck_rho = r.neck_rho;
    out->nonfinite = r.nonfinite;
}

int lbm_diagnostics(lbm_ctx *c, lbm_diag *out) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    DiagRecord r;
    hipError_t e = launch_diag(lattice_ref(c, c->cur), c->axis, c->partials, c->slices, c->latest, c->step,
                               nullptr, 0, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&r, c->latest, sizeof(r), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "lbm_diagnostics");
    to_public(r, out);
    if (r.nonfinite > 0)
        return fail(LBM_ERR_DIVERGED, "%lld nodes non-finite or with rho <= 0 at step %lld",
                    (long long)r.nonfinite, (long long)r.step);
    return LBM_OK;
}

static_assert(sizeof(lbm_droplet) == sizeof(DropletEntry) &&
                  offsetof(lbm_droplet, volume) == offsetof(DropletEntry, volume) &&
                  offsetof(lbm_droplet, mass) == offsetof(DropletEntry, mass) &&
                  offsetof(lbm_droplet, first_node) == offsetof(DropletEntry, first_node),
              "lbm_droplet mirrors the device table entry");

int lbm_droplets(lbm_ctx *c, double rho_mid, lbm_droplet *out, int32_t max_out, int64_t *count) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!count) return fail(LBM_ERR_INVALID_ARG, "count is NULL");
    if (max_out < 0) return fail(LBM_ERR_INVALID_ARG, "max_out must be >= 0");
    if (max_out > 0 && !out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    if (!std::isfinite(rho_mid)) return fail(LBM_ERR_INVALID_ARG, "rho_mid must be finite");
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    const int64_t n = int64_t(c->p.nx) * c->p.ny * c->p.nz;
    // Work arrays in the spare lattice (19 n b >= 38 n bytes): rho and mass
    // (8 n each), parent and volume (4 n each), two counters.
    char *w0 = static_cast<char *>(c->lat[c->cur ^ 1]);
    if (size_t(24 * n + 8) > c->lay.lat_bytes) return fail(LBM_ERR_INVALID_ARG, "spare lattice too small");
    DropletScratch w;
    w.rho = reinterpret_cast<double *>(w0);
    w.mass = reinterpret_cast<double *>(w0 + 8 * n);
    w.parent = reinterpret_cast<int32_t *>(w0 + 16 * n);
    w.vol = reinterpret_cast<int32_t *>(w0 + 20 * n);
    w.counters = reinterpret_cast<int32_t *>(w0 + 24 * n);
    int32_t ncomp = 0;
    hipError_t e = launch_droplets_label(lattice_ref(c, c->cur), rho_mid, w, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&ncomp, w.counters, sizeof(ncomp), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<DropletEntry> table(size_t(ncomp > 0 ? ncomp : 0));
    if (e == hipSuccess && ncomp > 0) {
        DropletEntry *d = nullptr;
        e = hipMalloc(&d, sizeof(DropletEntry) * size_t(ncomp));
        if (e == hipSuccess) e = launch_droplets_table(w, int(n), d, ncomp, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(table.data(), d, sizeof(DropletEntry) * size_t(ncomp), hipMemcpyDeviceToHost,
                               c->stream);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = e2;
        if (d) (void)hipFree(d);
    }
    if (e != hipSuccess) return device_fail(c, e, "lbm_droplets");
    std::sort(table.begin(), table.end(), [](const DropletEntry &a, const DropletEntry &b) {
        return a.volume != b.volume ? a.volume > b.volume : a.first_node < b.first_node;
    });
    *count = ncomp;
    const int64_t k = ncomp < max_out ? ncomp : max_out;
    for (int64_t i = 0; i < k; ++i) {
        out[i].volume = table[i].volume;
        out[i].mass = table[i].mass;
        out[i].first_node = table[i].first_node;
    }
    return LBM_OK;
}

int lbm_set_axis(lbm_ctx *c, int32_t axis) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (axis < 0 || axis > 2) return fail(LBM_ERR_INVALID_ARG, "axis must be 0, 1 or 2");
    c->axis = axis;
    return LBM_OK;
}

int lbm_record_diag(lbm_ctx *c) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    DiagRecord *slot = c->ring + (c->ring_written % LBM_DIAG_RING);
    hipError_t e = launch_diag(lattice_ref(c, c->cur), c->axis, c->partials, c->slices, slot, c->step, nullptr, 0,
                               c->stream);
    if (e != hipSuccess) return device_fail(c, e, "lbm_record_diag");
    c->ring_written += 1;
    return LBM_OK;
}

int lbm_read_diag_history(lbm_ctx *c, lbm_diag *out, int32_t max, int32_t *count) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!count || (max > 0 && !out) || max < 0) return fail(LBM_ERR_INVALID_ARG, "bad output arguments");
    int64_t first = c->ring_read;
    if (c->ring_written - first > LBM_DIAG_RING) first = c->ring_written - LBM_DIAG_RING;
    int64_t avail = c->ring_written - first;
    if (avail > max) avail = max;
    std::vector<DiagRecord> host(LBM_DIAG_RING);
    hipError_t e = hipMemcpyAsync(host.data(), c->ring, sizeof(DiagRecord) * LBM_DIAG_RING,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "lbm_read_diag_history");
    for (int64_t i = 0; i < avail; ++i) to_public(host[(first + i) % LBM_DIAG_RING], &out[i]);
    c->ring_read = first + avail;
    *count = int32_t(avail);
    return LBM_OK;
}

int lbm_get_step(const lbm_ctx *c, int64_t *step) {
    if (!c || !step) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
    *step = c->step;
    return LBM_OK;
}

int lbm_set_step(lbm_ctx *c, int64_t step) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (step < 0) return fail(LBM_ERR_INVALID_ARG, "step must be >= 0");
    c->step = step;
    return LBM_OK;
}

int lbm_set_launch(lbm_ctx *c, const lbm_launch *l) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    st = check_launch(l, c->p.storage);
    if (st != LBM_OK) return st;
    if (c->mrt.on && !tile_has_mrt(find_tile(l->tile_x, l->tile_y)))
        return fail(LBM_ERR_UNSUPPORTED, "the MRT collision runs on the run-time tiles (tile_x = 0) only");
    c->launch = *l;
    c->tile_index = find_tile(l->tile_x, l->tile_y);
    return LBM_OK;
}

int lbm_get_launch(const lbm_ctx *c, lbm_launch *l) {
    if (!c || !l) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
    *l = c->launch;
    return LBM_OK;
}

int lbm_list_tiles(lbm_launch *out, int32_t max, int32_t *count) {
    if (!count || (max > 0 && !out) || max < 0) return fail(LBM_ERR_INVALID_ARG, "bad output arguments");
    const int n = num_tiles();
    for (int i = 0; i < n && i < max; ++i) {
        tile_shape(i, &out[i].tile_x, &out[i].tile_y);
        out[i].zchunk = 0;
    }
    *count = n;
    return LBM_OK;
}

int lbm_default_launch(const lbm_params *p, lbm_launch *out, int32_t *tile_w, int32_t *tile_h) {
    const int st = validate_params(p);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    *out = default_launch(p);
    int tw = 0, th = 0;
    tile_dims(*out, p->nx, p->ny, &tw, &th);
    if (tile_w) *tile_w = tw;
    if (tile_h) *tile_h = th;
    return LBM_OK;
}

int lbm_lattice_layout(const lbm_params *p, int32_t *rows_per_record, int64_t *lattice_bytes) {
    const int st = validate_params(p);
    if (st != LBM_OK) return st;
    const Layout L = layout_of(p);
    if (rows_per_record) *rows_per_record = int32_t(1) << L.rec_shift;
    if (lattice_bytes) *lattice_bytes = int64_t(L.lat_bytes);
    return LBM_OK;
}

int lbm_autotune(lbm_ctx *c, int32_t steps_per_candidate, lbm_launch *best, double *best_mlups) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!c->initialized) return fail(LBM_ERR_STATE, "lattice not initialised");
    if (steps_per_candidate < 1) return fail(LBM_ERR_INVALID_ARG, "steps_per_candidate must be >= 1");
    // Candidates: the context's launch, the default launch, then every
    // compiled tile with z chunks of 1 to 256 planes.
    std::vector<lbm_launch> cands{c->launch, default_launch(&c->p)};
    const int zcs[] = {1, 2, 4, 8, 16, 32, 64, 128, 256};
    for (int ti = 0; ti < num_tiles(); ++ti) {
        lbm_launch l;
        tile_shape(ti, &l.tile_x, &l.tile_y);
        if (l.tile_x > 2 * c->p.nx && l.tile_x > 32) continue;  // mostly idle lanes
        for (int zc : zcs) {
            if (zc > c->p.nz && zc != zcs[0]) break;
            l.zchunk = zc;
            cands.push_back(l);
        }
    }
    // Each candidate is timed in the loop lbm_step runs: steps alternate
    // between the two lattices (an even number, so every candidate starts
    // and ends on the current one).  The state is saved to a temporary copy
    // first and restored at the end.
    const int pairs = (steps_per_candidate + 1) / 2;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *saved = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMalloc(&saved, c->lay.lat_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(saved, c->lat[c->cur], c->lay.lat_bytes, hipMemcpyDeviceToDevice, c->stream);
    double best_t = INFINITY;
    lbm_launch bl = c->launch;
    const double nodes = double(c->p.nx) * c->p.ny * c->p.nz;
    for (const lbm_launch &l : cands) {
        if (e != hipSuccess) break;
        const int ti = find_tile(l.tile_x, l.tile_y);
        if (ti < 0 || (c->mrt.on && !tile_has_mrt(ti)) || !tile_has_storage(ti, c->p.storage)) continue;
        const StepArgs A = step_args(c, l, c->cur), B = step_args(c, l, c->cur ^ 1);
        auto two_steps = [&]() {
            hipError_t r = launch_step(ti, c->p.storage, A, c->stream);
            if (r == hipSuccess) r = launch_step(ti, c->p.storage, B, c->stream);
            return r;
        };
        e = two_steps();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int s = 0; s < pairs && e == hipSuccess; ++s) e = two_steps();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        const double t = ms / (2.0 * pairs);
        if (t < best_t) {
            best_t = t;
            bl = l;
        }
    }
    if (saved) {
        hipError_t r = hipMemcpyAsync(c->lat[c->cur], saved, c->lay.lat_bytes, hipMemcpyDeviceToDevice, c->stream);
        if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = r;
        (void)hipFree(saved);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return device_fail(c, e, "lbm_autotune");
    c->launch = bl;
    c->tile_index = find_tile(bl.tile_x, bl.tile_y);
    cache_store(tune_key(&c->p), bl);
    if (best) *best = bl;
    if (best_mlups) *best_mlups = nodes / (best_t * 1e-3) / 1e6;
    return LBM_OK;
}

int lbm_set_graph_chunk(lbm_ctx *c, int32_t chunk_steps) {
    int st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (chunk_steps < 0 || (chunk_steps & 1)) return fail(LBM_ERR_INVALID_ARG, "chunk_steps must be even and >= 0");
    if (chunk_steps > 0 && !c->stream)
        return fail(LBM_ERR_UNSUPPORTED, "graph capture needs a non-null stream");
    release_graph(c);
    c->graph_chunk = chunk_steps;
    return LBM_OK;
}

int lbm_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src) return fail(LBM_ERR_INVALID_ARG, "NULL pointer");
    if (bytes % 16) return fail(LBM_ERR_INVALID_ARG, "bytes must be a multiple of 16");
    hipError_t e = launch_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, "lbm_device_copy: %s", hipGetErrorString(e));
    return LBM_OK;
}

}  // extern "C"

// ===========================================================================
// Batched form.
//
// Workspace: [case table][work items][frozen flags][diag records]
//            [diag partials][slice maxima][lattice pairs of every case].
// One launch per step processes the flat item list of all cases; a case's
// frozen flag (set by the diagnostics on a non-finite or non-positive
// density, to 1 + the lattice index current at that moment) makes its items
// return immediately, so its state stays as it was when it was frozen.

struct lbm_batch {
    int n;
    std::vector<lbm_params> p;
    std::vector<Layout> lay;
    std::vector<size_t> lat_off;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    BatchCase *d_cases;
    int4 *d_items;
    int32_t *d_frozen;
    DiagRecord *d_records;
    DiagPartial *d_partials;
    unsigned long long *d_slices;
    size_t item_capacity;
    int nitems;
    int parity;
    int64_t step;
    int check_every;
    int64_t since_check;
    bool initialized;
    bool poisoned;
    lbm_launch launch;
    int tile_index;
    int graph_chunk;
    hipGraphExec_t gexec;
    lbm_launch graph_launch;
    int graph_parity;
    // Frozen cases are dropped from the item list once the host has seen
    // their flags: h_frozen (pinned) receives a copy after each check,
    // ev_frozen marks its arrival, dropped[i] = case i has no items.
    int32_t *h_frozen;
    hipEvent_t ev_frozen;
    bool frozen_pending;
    std::vector<uint8_t> dropped;
    uint32_t *counter;  // device step counter, as in lbm_ctx
    uint32_t dstep;
    // > 0: per-case z chunks sized so that every work item costs about the
    // same and the launch holds about `rounds` times as many items as the
    // device runs at once; 0: every case uses the launch's zchunk.
    int rounds;
};

namespace {

constexpr int kBatchMinZchunk = 4;

int64_t items_for(const lbm_params &p, int tx, int ty, int zc) {
    lbm_launch l;
    l.tile_x = tx;
    l.tile_y = ty;
    l.zchunk = zc;
    tile_dims(l, p.nx, p.ny, &tx, &ty);
    const int64_t t = int64_t((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
    const int z = zc < p.nz ? zc : p.nz;
    return t * ((p.nz + z - 1) / z);
}

struct BatchLayout {
    size_t off_cases, off_items, off_frozen, off_records, off_partials, off_slices, off_counter, off_lat, total;
    size_t item_capacity;
    int max_parts, max_slices;
    std::vector<Layout> lay;
    std::vector<size_t> lat_off;
};

BatchLayout batch_layout(int n, const lbm_params *p) {
    BatchLayout B;
    B.item_capacity = 0;
    B.max_parts = 1;
    B.max_slices = 1;
    for (int t = 0; t < num_tiles(); ++t) {
        int tx, ty;
        tile_shape(t, &tx, &ty);
        size_t cnt = 0;
        for (int i = 0; i < n; ++i) cnt += size_t(items_for(p[i], tx, ty, kBatchMinZchunk));
        // the launch list pads each XCD's share to the longest one (batch_upload)
        cnt = 8 * cnt + 8;
        if (cnt > B.item_capacity) B.item_capacity = cnt;
    }
    for (int i = 0; i < n; ++i) {
        B.lay.push_back(layout_of(&p[i]));
        if (B.lay.back().nparts > B.max_parts) B.max_parts = B.lay.back().nparts;
        if (B.lay.back().nslices > B.max_slices) B.max_slices = B.lay.back().nslices;
    }
    size_t off = 0;
    B.off_cases = off;
    off += align_up(sizeof(BatchCase) * n, 256);
    B.off_items = off;
    off += align_up(sizeof(int4) * B.item_capacity, 256);
    B.off_frozen = off;
    off += align_up(sizeof(int32_t) * n, 256);
    B.off_records = off;
    off += align_up(sizeof(DiagRecord) * n, 256);
    B.off_partials = off;
    off += align_up(sizeof(DiagPartial) * B.max_parts, 256);
    B.off_slices = off;
    off += align_up(sizeof(unsigned long long) * B.max_slices, 256);
    B.off_counter = off;
    off += 256;
    B.off_lat = off;
    for (int i = 0; i < n; ++i) {
        B.lat_off.push_back(off);
        off += 2 * B.lay[i].lat_bytes;
    }
    B.total = off;
    return B;
}

int validate_batch(int n, const lbm_params *p) {
    if (n < 1) return fail(LBM_ERR_INVALID_ARG, "a batch needs at least one case");
    if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
    for (int i = 0; i < n; ++i) {
        int st = validate_params(&p[i]);
        if (st != LBM_OK) {
            const std::string m = g_err;
            return fail(st, "case %d: %s", i, m.c_str());
        }
        if (p[i].storage != p[0].storage)
            return fail(LBM_ERR_INVALID_ARG, "case %d: all cases must share one storage kind", i);
    }
    return LBM_OK;
}

int batch_check(const lbm_batch *b) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (b->poisoned) return fail(LBM_ERR_STATE, "batch is poisoned by an earlier device error");
    return LBM_OK;
}

int batch_device_fail(lbm_batch *b, hipError_t e, const char *what) {
    b->poisoned = true;
    return fail(LBM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void *case_lat(const lbm_batch *b, int i, int which) {
    return b->ws + b->lat_off[i] + (which ? b->lay[i].lat_bytes : 0);
}

LatticeRef batch_ref(const lbm_batch *b, int i, int which) {
    LatticeRef L;
    L.lat = case_lat(b, i, which);
    L.nx = b->p[i].nx;
    L.ny = b->p[i].ny;
    L.nz = b->p[i].nz;
    L.storage = b->p[i].storage;
    L.pop_stride = b->lay[i].S;
    L.row_stride = b->lay[i].R;
    L.plane_stride = b->lay[i].P;
    L.rec_shift = b->lay[i].rec_shift;
    L.rho_ref = is_shifted(b->p[i].storage) ? b->p[i].rho_ref : 0.0;
    L.frozen = b->d_frozen + i;
    L.pair[0] = case_lat(b, i, 0);
    L.pair[1] = case_lat(b, i, 1);
    return L;
}

// Rebuild the device case table and item list for the current launch shape.
//
// Work items are (case, tile, z chunk) triples of the cases still running.
// The hardware hands workgroup b to XCD b mod 8, and each XCD runs its
// workgroups in launch order, so the list is built per XCD and interleaved:
//  - the items, in (case, chunk, tile) order, are cut into 8 runs of equal
//    estimated cost, one per XCD: neighbouring tiles and chunks of a case,
//    whose ring and boundary planes overlap, meet in one L2, and every XCD
//    has the same amount of work;
//  - within a run the items go longest first, so that each XCD ends on its
//    shortest items and the step's tail is short;
//  - runs shorter than the longest are padded with empty items (case -1).
// Cost of an item: (planes + 2) x (tile nodes + ring nodes), the two extra
// planes being the chunk's boundary gathers.
hipError_t batch_upload(lbm_batch *b) {
    std::vector<BatchCase> cases(b->n);
    struct Item {
        int4 it;
        double cost;
    };
    std::vector<Item> all;
    const lbm_launch &l = b->launch;
    // z chunk per case: uniform, or (rounds > 0) about rounds x slots items
    // of equal cost, cost per plane = tile + ring nodes
    std::vector<int> zc_case(b->n, l.zchunk);
    if (b->rounds > 0) {
        double plane_cost = 0;
        std::vector<double> area(b->n, 0.0);
        std::vector<int64_t> tiles(b->n, 0);
        for (int i = 0; i < b->n; ++i) {
            if (b->dropped[i]) continue;
            int tw, th;
            tile_dims(l, b->p[i].nx, b->p[i].ny, &tw, &th);
            tiles[i] = int64_t((b->p[i].nx + tw - 1) / tw) * ((b->p[i].ny + th - 1) / th);
            area[i] = double(tw) * th + 2.0 * (tw + 2) + 2.0 * th;
            plane_cost += double(tiles[i]) * b->p[i].nz * area[i];
        }
        int slots = launch_slots(b->tile_index, b->p[0].storage);
        if (slots <= 0) slots = 512;
        const double per_item = plane_cost / (double(b->rounds) * slots);
        for (int i = 0; i < b->n; ++i) {
            if (b->dropped[i]) continue;
            const int nz = b->p[i].nz;
            int zc = int(per_item / area[i] + 0.5);
            zc = std::max(kBatchMinZchunk, std::min(zc, nz));
            const int nch = (nz + zc - 1) / zc;
            zc_case[i] = std::max(std::min(kBatchMinZchunk, nz), (nz + nch - 1) / nch);
        }
    }
    for (int i = 0; i < b->n; ++i) {
        StepArgs A;
        A.src = nullptr;
        A.dst = nullptr;
        A.nx = b->p[i].nx;
        A.ny = b->p[i].ny;
        A.nz = b->p[i].nz;
        tile_dims(l, A.nx, A.ny, &A.tile_w, &A.tile_h);
        A.tiles_x = (A.nx + A.tile_w - 1) / A.tile_w;
        A.tiles_y = (A.ny + A.tile_h - 1) / A.tile_h;
        A.zchunk = zc_case[i] < A.nz ? zc_case[i] : A.nz;
        A.nchunks = (A.nz + A.zchunk - 1) / A.zchunk;
        A.pop_stride = b->lay[i].S;
        A.row_stride = b->lay[i].R;
        A.plane_stride = b->lay[i].P;
        A.rec_shift = b->lay[i].rec_shift;
        A.tau = b->p[i].tau;
        A.G = b->p[i].G;
        A.rho0 = b->p[i].rho0;
        A.rho_ref = is_shifted(b->p[i].storage) ? b->p[i].rho_ref : 0.0;
        A.mrt = MrtParams{};  // the batched form uses BGK
        cases[i].args = A;
        cases[i].lat[0] = case_lat(b, i, 0);
        cases[i].lat[1] = case_lat(b, i, 1);
        if (b->dropped[i]) continue;  // frozen: its workgroups would only exit
        const double area = double(A.tile_w) * A.tile_h + 2.0 * (A.tile_w + 2) + 2.0 * A.tile_h;
        for (int c = 0; c < A.nchunks; ++c) {
            const int planes = std::min(A.zchunk, A.nz - c * A.zchunk);
            for (int t = 0; t < A.tiles_x * A.tiles_y; ++t)
                all.push_back(Item{make_int4(i, t, c, 0), (planes + 2) * area});
        }
    }
    double total = 0;
    for (const Item &it : all) total += it.cost;
    constexpr int kXcd = 8;
    std::vector<std::vector<Item>> run(kXcd);
    double acc = 0;
    for (const Item &it : all) {
        int x = int(acc / total * kXcd);  // the run this item's cost midpoint falls in
        acc += it.cost;
        x = std::min(std::max(x, 0), kXcd - 1);
        run[x].push_back(it);
    }
    size_t longest = 0;
    for (auto &r : run) {
        std::stable_sort(r.begin(), r.end(), [](const Item &p, const Item &q) { return p.cost > q.cost; });
        longest = std::max(longest, r.size());
    }
    std::vector<int4> items;
    items.reserve(kXcd * longest);
    for (size_t j = 0; j < longest && !all.empty(); ++j)
        for (int x = 0; x < kXcd; ++x) items.push_back(j < run[x].size() ? run[x][j].it : make_int4(-1, 0, 0, 0));
    if (items.size() > b->item_capacity) return hipErrorInvalidValue;  // zchunk below the sized minimum
    b->nitems = int(items.size());
    hipError_t e = hipMemcpyAsync(b->d_cases, cases.data(), sizeof(BatchCase) * b->n, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpyAsync(b->d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // host vectors die here
    return e;
}

hipError_t batch_check_divergence(lbm_batch *b, DiagRecord *records) {
    for (int i = 0; i < b->n; ++i) {
        hipError_t e = launch_diag(batch_ref(b, i, b->parity), 2, b->d_partials, b->d_slices, records + i,
                                   b->step, b->d_frozen + i, b->parity + 1, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t batch_plain(lbm_batch *b, int64_t n) {
    for (int64_t s = 0; s < n; ++s) {
        if (b->nitems > 0) {  // no items: every case is frozen
            hipError_t e = launch_step_batch(b->tile_index, b->p[0].storage, b->d_cases, b->d_items, b->nitems,
                                             b->d_frozen, b->parity, b->counter, uint32_t(b->step) - b->dstep,
                                             b->stream);
            if (e != hipSuccess) return e;
        }
        b->parity ^= 1;
        b->step += 1;
    }
    return hipSuccess;
}

void batch_release_graph(lbm_batch *b) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
}

hipError_t batch_build_graph(lbm_batch *b) {
    batch_release_graph(b);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int s = 0; s < b->graph_chunk && e == hipSuccess; ++s)
        e = launch_step_batch(b->tile_index, b->p[0].storage, b->d_cases, b->d_items, b->nitems, b->d_frozen,
                              s & 1, b->counter, uint32_t(s), b->stream);
    if (e == hipSuccess) e = launch_counter(b->counter, uint32_t(b->graph_chunk), true, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    b->graph_launch = b->launch;
    return e;
}

// Drop the cases the last copied flags show frozen from the item list (the
// upload synchronises the stream; it happens once per newly frozen set).
hipError_t batch_compact(lbm_batch *b) {
    b->frozen_pending = false;
    bool changed = false;
    for (int i = 0; i < b->n; ++i)
        if (b->h_frozen[i] != 0 && !b->dropped[i]) {
            b->dropped[i] = 1;
            changed = true;
        }
    if (!changed) return hipSuccess;
    batch_release_graph(b);
    return batch_upload(b);
}

// After a divergence check has been enqueued: take in the flags of the
// previous check (waiting for the device to reach it, so the host runs at
// most one check interval ahead), then queue the copy of the new flags.
hipError_t batch_after_check(lbm_batch *b) {
    hipError_t e = hipSuccess;
    if (b->frozen_pending) {
        e = hipEventSynchronize(b->ev_frozen);
        if (e == hipSuccess) e = batch_compact(b);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_frozen, b->d_frozen, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_frozen, b->stream);
    if (e == hipSuccess) b->frozen_pending = true;
    return e;
}

lbm_launch batch_default_launch(int n, const lbm_params *p) {
    (void)n;
    lbm_launch l;
    l.tile_x = 0;  // each case gets its own full-row tile shape
    // Measured on MI355X over the 51 live cases of the 64-ligament batch
    // (FP32, whole-row tiles with their ghost ring): 1024-thread tiles with
    // z chunks of 5 planes 0.779 ms per step, 8 planes 0.789, 16 planes
    // 0.825; 512-thread tiles 0.796 (5 planes) to 0.825 (16).  FP64 keeps 512
    // threads (its kernel spills with 1024).
    l.tile_y = p[0].storage == LBM_F64 ? 512 : 1024;
    l.zchunk = 5;
    return l;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t ncases, const lbm_params *p) {
    if (validate_batch(ncases, p) != LBM_OK) return 0;
    return batch_layout(ncases, p).total;
}

int lbm_batch_create(int32_t ncases, const lbm_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream,
                     lbm_batch **out) {
    int st = validate_batch(ncases, p);
    if (st != LBM_OK) return st;
    if (!out || !d_workspace) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
        return fail(LBM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    BatchLayout B = batch_layout(ncases, p);
    if (ws_bytes < B.total)
        return fail(LBM_ERR_BUFFER_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, B.total);
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    b->n = ncases;
    b->p.assign(p, p + ncases);
    b->lay = B.lay;
    b->lat_off = B.lat_off;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char *>(d_workspace);
    b->ws_bytes = ws_bytes;
    b->d_cases = reinterpret_cast<BatchCase *>(b->ws + B.off_cases);
    b->d_items = reinterpret_cast<int4 *>(b->ws + B.off_items);
    b->d_frozen = reinterpret_cast<int32_t *>(b->ws + B.off_frozen);
    b->d_records = reinterpret_cast<DiagRecord *>(b->ws + B.off_records);
    b->d_partials = reinterpret_cast<DiagPartial *>(b->ws + B.off_partials);
    b->d_slices = reinterpret_cast<unsigned long long *>(b->ws + B.off_slices);
    b->counter = reinterpret_cast<uint32_t *>(b->ws + B.off_counter);
    b->dstep = 0;
    b->rounds = 0;
    b->item_capacity = B.item_capacity;
    b->parity = 0;
    b->step = 0;
    b->check_every = 1000;
    b->since_check = 0;
    b->initialized = false;
    b->poisoned = false;
    b->graph_chunk = 0;
    b->gexec = nullptr;
    b->launch = batch_default_launch(ncases, p);
    b->tile_index = find_tile(b->launch.tile_x, b->launch.tile_y);
    b->h_frozen = nullptr;
    b->ev_frozen = nullptr;
    b->frozen_pending = false;
    b->dropped.assign(ncases, 0);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&b->h_frozen), sizeof(int32_t) * ncases,
                                 hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_frozen, hipEventDisableTiming);
    if (e == hipSuccess) e = launch_fill_u64(b->d_slices, B.max_slices, 0ull, b->stream);
    if (e == hipSuccess) e = launch_counter(b->counter, 0u, false, b->stream);
    if (e == hipSuccess) e = batch_upload(b);
    if (e != hipSuccess) {
        if (b->ev_frozen) (void)hipEventDestroy(b->ev_frozen);
        if (b->h_frozen) (void)hipHostFree(b->h_frozen);
        delete b;
        return fail(LBM_ERR_DEVICE, "lbm_batch_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch *b) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (b->gexec) (void)hipStreamSynchronize(b->stream);
    batch_release_graph(b);
    if (b->ev_frozen) (void)hipEventDestroy(b->ev_frozen);
    if (b->h_frozen) (void)hipHostFree(b->h_frozen);
    delete b;
    return LBM_OK;
}

int lbm_batch_init(lbm_batch *b, const lbm_ligament *specs) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (!specs) return fail(LBM_ERR_INVALID_ARG, "specs is NULL");
    std::vector<LigamentArgs> args(b->n);
    for (int i = 0; i < b->n; ++i) {
        const lbm_ligament *g = &specs[i];
        if (g->axis < 0 || g->axis > 2 || !(g->R0 > 0) || !(g->wavelength > 0) || !(g->width > 0) ||
            !(g->noise_amp >= 0) || !isfinite(g->amp_rel) || !isfinite(g->c1) || !isfinite(g->c2))
            return fail(LBM_ERR_INVALID_ARG, "case %d: invalid ligament spec", i);
        LigamentArgs &a = args[i];
        a.axis = g->axis;
        a.R0 = g->R0;
        a.amp_rel = g->amp_rel;
        a.wavelength = g->wavelength;
        a.c1 = g->c1;
        a.c2 = g->c2;
        a.width = g->width;
        a.rho_l = g->rho_l;
        a.rho_v = g->rho_v;
        a.noise_amp = g->noise_amp;
        a.seed = g->seed;
        if (!(a.rho_l > 0) || !(a.rho_v > 0)) {
            st = check_coexistence_args(b->p[i].G, b->p[i].tau, b->p[i].psi, b->p[i].rho0);
            if (st != LBM_OK) {
                const std::string m = g_err;
                return fail(st, "case %d: %s", i, m.c_str());
            }
        }
    }
    // Densities of the cases that need them: their flat-interface runs advance
    // together, one workgroup each.  A run that diverges (the flat interface
    // itself is unstable at that G and tau) leaves its case frozen from the
    // start, with non-finite densities its diagnostics report.
    std::vector<CoexRun> runs;
    std::vector<int> need;
    for (int i = 0; i < b->n; ++i)
        if (!(args[i].rho_l > 0) || !(args[i].rho_v > 0)) {
            runs.emplace_back(b->p[i].G, b->p[i].tau, b->p[i].rho0, MrtParams{});
            need.push_back(i);
        }
    if (!runs.empty()) {
        const hipError_t ce = run_coexistence(runs);
        if (ce != hipSuccess) return fail(LBM_ERR_DEVICE, "lbm_batch_init: %s", hipGetErrorString(ce));
        for (size_t k = 0; k < runs.size(); ++k) {
            LigamentArgs &a = args[size_t(need[k])];
            a.rho_l = runs[k].diverged ? NAN : runs[k].bl;
            a.rho_v = runs[k].diverged ? NAN : runs[k].bv;
        }
    }
    hipError_t e = hipSuccess;
    std::vector<int32_t> flags(b->n, 0);
    for (int i = 0; i < b->n; ++i) flags[i] = isnan(args[i].rho_l) ? 1 : 0;  // state in lattice 0
    e = hipMemcpyAsync(b->d_frozen, flags.data(), sizeof(int32_t) * b->n, hipMemcpyHostToDevice, b->stream);
    for (int i = 0; i < b->n && e == hipSuccess; ++i) e = launch_init_ligament(batch_ref(b, i, 0), args[i], b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) {
        // a new state: item lists of every case, minus those frozen from the start
        b->frozen_pending = false;
        for (int i = 0; i < b->n; ++i) b->dropped[i] = uint8_t(flags[i] != 0);
        batch_release_graph(b);
        e = batch_upload(b);
    }
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_init");
    b->parity = 0;
    b->step = 0;
    b->since_check = 0;
    b->initialized = true;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (nsteps < 0) return fail(LBM_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!b->initialized) return fail(LBM_ERR_STATE, "batch not initialised");
    hipError_t e = hipSuccess;
    if (b->frozen_pending) {  // flags of the last check already here: drop frozen cases now
        const hipError_t q = hipEventQuery(b->ev_frozen);
        if (q == hipSuccess) e = batch_compact(b);
        else if (q != hipErrorNotReady) e = q;
    }
    int64_t left = nsteps;
    while (e == hipSuccess && left > 0) {
        // run up to the next divergence check
        int64_t run = b->check_every - b->since_check;
        if (run > left) run = left;
        int64_t r = run;
        if (b->graph_chunk > 0 && r >= b->graph_chunk && b->nitems > 0) {
            if (b->parity == 1) {
                e = batch_plain(b, 1);
                r -= 1;
            }
            if (e == hipSuccess && (!b->gexec || memcmp(&b->graph_launch, &b->launch, sizeof(lbm_launch)) != 0))
                e = batch_build_graph(b);
            if (e == hipSuccess && b->dstep != uint32_t(b->step)) {
                e = launch_counter(b->counter, uint32_t(b->step), false, b->stream);
                b->dstep = uint32_t(b->step);
            }
            while (e == hipSuccess && r >= b->graph_chunk) {
                e = hipGraphLaunch(b->gexec, b->stream);
                b->step += b->graph_chunk;
                b->dstep += uint32_t(b->graph_chunk);
                r -= b->graph_chunk;
            }
        }
        if (e == hipSuccess) e = batch_plain(b, r);
        left -= run;
        b->since_check += run;
        if (e == hipSuccess && b->since_check >= b->check_every) {
            e = batch_check_divergence(b, b->d_records);
            if (e == hipSuccess) e = batch_after_check(b);
            b->since_check = 0;
        }
    }
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_step");
    return LBM_OK;
}

int lbm_batch_diagnostics(lbm_batch *b, lbm_diag *out) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    if (!b->initialized) return fail(LBM_ERR_STATE, "batch not initialised");
    std::vector<DiagRecord> rec(b->n);
    hipError_t e = batch_check_divergence(b, b->d_records);
    if (e == hipSuccess)
        e = hipMemcpyAsync(rec.data(), b->d_records, sizeof(DiagRecord) * b->n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_frozen, b->d_frozen, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = batch_compact(b);
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_diagnostics");
    for (int i = 0; i < b->n; ++i) to_public(rec[i], &out[i]);
    return LBM_OK;
}

int lbm_batch_get_fields(lbm_batch *b, int32_t index, uint32_t mask, double *rho, double *u, double *force,
                         double *pop, int32_t on_device) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (index < 0 || index >= b->n) return fail(LBM_ERR_INVALID_ARG, "case index %d out of range", index);
    if (!b->initialized) return fail(LBM_ERR_STATE, "batch not initialised");
    int32_t fz = 0;
    hipError_t e = hipMemcpyAsync(&fz, b->d_frozen + index, sizeof(fz), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_get_fields");
    LatticeRef L = batch_ref(b, index, fz ? fz - 1 : b->parity);
    L.frozen = nullptr;
    st = get_fields_impl(nullptr, L, b->p[index], b->stream, mask, rho, u, force, pop, on_device);
    if (st == LBM_ERR_DEVICE) b->poisoned = true;
    return st;
}

int lbm_batch_set_launch(lbm_batch *b, const lbm_launch *l) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    st = check_launch(l, b->p[0].storage);
    if (st != LBM_OK) return st;
    if (l->zchunk < kBatchMinZchunk) return fail(LBM_ERR_INVALID_ARG, "batched zchunk must be >= %d", kBatchMinZchunk);
    b->launch = *l;
    b->tile_index = find_tile(l->tile_x, l->tile_y);
    b->rounds = 0;
    hipError_t e = batch_upload(b);
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_set_launch");
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch *b, int32_t steps_per_candidate, lbm_launch *best, double *best_mlups) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (!b->initialized) return fail(LBM_ERR_STATE, "batch not initialised");
    if (steps_per_candidate < 1) return fail(LBM_ERR_INVALID_ARG, "steps_per_candidate must be >= 1");
    // Candidates: every tile with uniform z chunks, and with equal-cost
    // chunks of 4 to 32 rounds (lbm_batch_set_chunking).  Short chunks
    // matter here: the batch's grids are narrow, so their workgroups are few
    // per case, and many short items balance the launch.
    struct Cand {
        lbm_launch l;
        int rounds;
    };
    std::vector<Cand> cands;
    const int zcs[] = {4, 5, 6, 8, 12, 16, 32, 64, 128};
    const int rounds[] = {4, 8, 16, 32};
    for (int ti = 0; ti < num_tiles(); ++ti) {
        if (!tile_has_storage(ti, b->p[0].storage)) continue;
        lbm_launch l;
        tile_shape(ti, &l.tile_x, &l.tile_y);
        for (int zc : zcs) {
            l.zchunk = zc;
            cands.push_back(Cand{l, 0});
        }
        l.zchunk = kBatchMinZchunk;
        for (int r : rounds) cands.push_back(Cand{l, r});
    }
    lbm_launch bl = b->launch;
    int brounds = b->rounds;
    double best_t = INFINITY;
    // Candidates are timed in the loop lbm_batch_step runs: launches that
    // alternate between the two lattices of every case (an even number).
    // The current lattices of the cases in the launch list are saved first
    // and restored at the end; frozen cases are not touched by the step.
    std::vector<int> live;
    size_t save_bytes = 0;
    for (int i = 0; i < b->n; ++i)
        if (!b->dropped[i]) {
            live.push_back(i);
            save_bytes += b->lay[i].lat_bytes;
        }
    std::vector<int32_t> fz(b->n, 0);
    const int pairs = (steps_per_candidate + 1) / 2;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    char *saved = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess && save_bytes) e = hipMalloc(reinterpret_cast<void **>(&saved), save_bytes);
    for (size_t k = 0, off = 0; k < live.size() && e == hipSuccess; off += b->lay[live[k]].lat_bytes, ++k)
        e = hipMemcpyAsync(saved + off, case_lat(b, live[k], b->parity), b->lay[live[k]].lat_bytes,
                           hipMemcpyDeviceToDevice, b->stream);
    // throughput is counted over the cases that are not frozen (frozen ones exit at once)
    if (e == hipSuccess)
        e = hipMemcpyAsync(fz.data(), b->d_frozen, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    double nodes = 0;
    for (int i = 0; i < b->n; ++i)
        if (fz[i] == 0) nodes += double(b->p[i].nx) * b->p[i].ny * b->p[i].nz;
    for (const Cand &c : cands) {
        if (e != hipSuccess) break;
        const int ti = find_tile(c.l.tile_x, c.l.tile_y);
        b->launch = c.l;
        b->tile_index = ti;
        b->rounds = c.rounds;
        e = batch_upload(b);
        if (e != hipSuccess) {
            if (e == hipErrorInvalidValue) e = hipSuccess;  // more items than the table holds
            continue;
        }
        auto two_steps = [&]() {
            hipError_t r = hipSuccess;
            if (b->nitems > 0)
                for (int q = 0; q < 2 && r == hipSuccess; ++q)
                    r = launch_step_batch(ti, b->p[0].storage, b->d_cases, b->d_items, b->nitems, b->d_frozen,
                                          b->parity ^ q, b->counter, uint32_t(b->step) - b->dstep, b->stream);
            return r;
        };
        e = two_steps();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int s = 0; s < pairs && e == hipSuccess; ++s) e = two_steps();
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        const double t = ms / (2.0 * pairs);
        if (t < best_t) {
            best_t = t;
            bl = c.l;
            brounds = c.rounds;
        }
    }
    if (saved) {
        hipError_t r = hipSuccess;
        for (size_t k = 0, off = 0; k < live.size() && r == hipSuccess; off += b->lay[live[k]].lat_bytes, ++k)
            r = hipMemcpyAsync(case_lat(b, live[k], b->parity), saved + off, b->lay[live[k]].lat_bytes,
                               hipMemcpyDeviceToDevice, b->stream);
        if (r == hipSuccess) r = hipStreamSynchronize(b->stream);
        if (e == hipSuccess) e = r;
        (void)hipFree(saved);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->launch = bl;
    b->tile_index = find_tile(bl.tile_x, bl.tile_y);
    b->rounds = brounds;
    if (e == hipSuccess) e = batch_upload(b);
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_autotune");
    batch_release_graph(b);
    if (best) *best = bl;
    if (best_mlups) *best_mlups = nodes / (best_t * 1e-3) / 1e6;
    return LBM_OK;
}

int lbm_batch_set_chunking(lbm_batch *b, int32_t rounds) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (rounds < 0) return fail(LBM_ERR_INVALID_ARG, "rounds must be >= 0");
    const int old = b->rounds;
    b->rounds = rounds;
    hipError_t e = batch_upload(b);
    if (e == hipErrorInvalidValue) {
        b->rounds = old;
        (void)batch_upload(b);
        return fail(LBM_ERR_INVALID_ARG, "chunking gives more work items than the workspace holds");
    }
    if (e != hipSuccess) return batch_device_fail(b, e, "lbm_batch_set_chunking");
    batch_release_graph(b);
    return LBM_OK;
}

int lbm_batch_set_graph_chunk(lbm_batch *b, int32_t chunk_steps) {
    int st = batch_check(b);
    if (st != LBM_OK) return st;
    if (chunk_steps < 0 || (chunk_steps & 1)) return fail(LBM_ERR_INVALID_ARG, "chunk_steps must be even and >= 0");
    if (chunk_steps > 0 && !b->stream) return fail(LBM_ERR_UNSUPPORTED, "graph capture needs a non-null stream");
    batch_release_graph(b);
    b->graph_chunk = chunk_steps;
    return LBM_OK;
}

}  // extern "C"
