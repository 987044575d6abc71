// Host runtime of the batched C ABI (include/gals.h, gals_batch_*): many
// independent 2D grids with sine stream-function fields, one launch per
// step over a work list of tiles, optional hipGraph capture of a whole
// advance, and a timing-based choice of the wave shape per grid-size class.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "batch_shape.h"
#include "gals_internal.h"

using namespace gals;

namespace {

int bfail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    gals::set_error_v(fmt, ap);
    va_end(ap);
    return code;
}

int bhip(hipError_t e, const char *what)
{
    return bfail(GALS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// wave shapes: nodes per wave along x (a wave covers 64/w rows), 0 = row-major
const unsigned kShapes[4] = {64u, 32u, 16u, 0u};

// Grid-size class of a problem by nodes per row.
int size_class(int n0) { return n0 <= 48 ? 0 : n0 <= 96 ? 1 : n0 <= 192 ? 2 : 3; }

// ---------------------------------------------------------------------------
// Tuned wave shapes per batch shape. The key is a 64-bit FNV-1a hash of the
// precision, the cross-derivative rule and every problem's cell counts in
// order; gals_batch_autotune records its choice under it, in this process
// and, when the environment variable GALS_TUNE_FILE names a file, as one
// line "key w0 w1 w2 w3" appended to that file; gals_batch_create starts a
// batch of a recorded shape with the recorded shapes (the file's last line
// for the key wins over earlier ones, the process's own record over the
// file).
// ---------------------------------------------------------------------------
std::mutex g_tune_mutex;
std::map<uint64_t, std::vector<unsigned>> g_tuned;

uint64_t fnv1a(uint64_t h, uint64_t v)
{
    for (int k = 0; k < 8; k++) {
        h ^= (v >> (8 * k)) & 0xffu;
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t shape_key(int prec, int mixed, int64_t nprob, const int64_t *ncell)
{
    uint64_t h = 14695981039346656037ull;
    h = fnv1a(h, uint64_t(prec));
    h = fnv1a(h, uint64_t(mixed));
    h = fnv1a(h, uint64_t(nprob));
    for (int64_t k = 0; k < 2 * nprob; k++) h = fnv1a(h, uint64_t(ncell[k]));
    return h;
}

bool valid_shape(unsigned w) { return w == 64u || w == 32u || w == 16u || w == 0u; }

// The recorded shapes for `key`, if any (the process's record first).
bool lookup_tuned(uint64_t key, unsigned out[4])
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
        for (int c = 0; c < 4; c++) out[c] = it->second[c];
        return true;
    }
    const char *path = getenv("GALS_TUNE_FILE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    unsigned long long k;
    unsigned w[4];
    while (fscanf(f, "%llx %u %u %u %u", &k, &w[0], &w[1], &w[2], &w[3]) == 5) {
        if (uint64_t(k) != key) continue;
        if (!(valid_shape(w[0]) && valid_shape(w[1]) && valid_shape(w[2]) && valid_shape(w[3])))
            continue;
        for (int c = 0; c < 4; c++) out[c] = w[c];
        found = true;
    }
    fclose(f);
    return found;
}

void record_tuned(uint64_t key, const unsigned w[4])
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuned[key] = std::vector<unsigned>(w, w + 4);
    const char *path = getenv("GALS_TUNE_FILE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%016llx %u %u %u %u\n", (unsigned long long)key, w[0], w[1], w[2], w[3]);
    fclose(f);
}

}  // namespace

struct gals_batch {
    int nprob = 0, prec = 0, mixed = 0, bc = 0, device = 0;
    std::vector<Geom> g;
    std::vector<int64_t> off, tab;
    std::vector<double> S;  // 16 per problem: summed amplitudes per (m, n)
    std::vector<char> vel_set;
    double period = 0.0;
    bool period_set = false;
    int64_t total_elems = 0, tab_elems = 0;
    int max_entries = 0;
    unsigned class_wx[4] = {64u, 64u, 64u, 64u};
    uint64_t shape_key = 0;  // key of the batch's shape for the tuning record
    unsigned blocks = 0;
    // device copies of the problem descriptors and the tile list
    void *d_probs = nullptr;
    void *d_probs64 = nullptr;
    TileRef *d_tiles = nullptr;
    unsigned ntiles = 0;
    bool dirty = true;
    // cached graph of one advance
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    void *gk_state = nullptr, *gk_ws = nullptr, *gk_stream = nullptr;
    double gk_t0 = 0, gk_dt = 0;
    int64_t gk_steps = -1;
};

namespace {

size_t es(const gals_batch *b) { return b->prec == GALS_F32 ? 4 : 8; }

// workspace: [ping-pong state copy | stream tables]
int64_t tab_offset(const gals_batch *b) { return round_up(b->total_elems * int64_t(es(b)), 256); }
size_t ws_bytes(const gals_batch *b)
{
    return size_t(tab_offset(b) + round_up(b->tab_elems * int64_t(es(b)), 256));
}

void drop_graph(gals_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->gk_steps = -1;
}

void free_device(gals_batch *b)
{
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_probs64 && b->d_probs64 != b->d_probs) (void)hipFree(b->d_probs64);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_probs = b->d_probs64 = nullptr;
    b->d_tiles = nullptr;
    b->ntiles = 0;
}

template <typename T>
void fill_prob(const gals_batch *b, int p, BatchProb<T> &P)
{
    memset(&P, 0, sizeof(P));
    P.g = b->g[p];
    int mmax = 0, nmax = 0;
    for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) {
            const double a = b->S[16 * p + 4 * m + n];
            const double kn = (n + 1) * M_PI;
            P.S[m][n] = T(a);
            P.SQ[m][n] = T(a * kn);
            P.SR[m][n] = T(a * kn * kn);
            if (a != 0.0) {
                mmax = m + 1 > mmax ? m + 1 : mmax;
                nmax = n + 1 > nmax ? n + 1 : nmax;
            }
        }
    P.kx = T(M_PI * mmax);
    P.ky = T(M_PI * nmax);
    P.off = b->off[p];
    P.tab = b->tab[p];
    P.wx = b->class_wx[size_class(P.g.n[0])];
    P.tiles_x = P.wx ? (unsigned(P.g.n[0]) + P.wx - 1u) / P.wx : 0u;
    P.inv_n0 = 1.0f / float(P.g.n[0]);
    if (packed_tail(P)) P.tiles_x = unsigned(P.g.n[0]) / 64u;  // full column groups only
}

// Tiles of problem P (4 waves of 64 lanes each).
unsigned tile_count(const BatchProb<double> &P)
{
    if (P.wx == 0u) return unsigned((P.g.nodes + 255) / 256);
    const unsigned rows = 4u * (64u / P.wx);
    const unsigned body = P.tiles_x * ((unsigned(P.g.n[1]) + rows - 1u) / rows);
    const uint64_t tail = uint64_t(packed_tail(P)) * uint64_t(P.g.n[1]);
    return body + unsigned((tail + 255u) / 256u);  // body == body_tiles(P) for 64 x 1 waves
}

// Upload descriptors and the tile list (synchronous; never inside a capture).
int upload(gals_batch *b)
{
    if (!b->dirty) return GALS_OK;
    drop_graph(b);
    free_device(b);
    std::vector<BatchProb<float>> pf;
    std::vector<BatchProb<double>> pd(b->nprob);
    std::vector<TileRef> tiles;
    if (b->prec == GALS_F32) pf.resize(b->nprob);
    for (int p = 0; p < b->nprob; p++) {
        fill_prob(b, p, pd[p]);
        if (b->prec == GALS_F32) fill_prob(b, p, pf[p]);
        const unsigned nt = tile_count(pd[p]);
        if (uint64_t(tiles.size()) + nt > (uint64_t(1) << 31))
            return bfail(GALS_EINVAL, "gals_batch: more than 2^31 tiles in one batch");
        const BatchProb<double> &P = pd[p];
        if (P.wx == 0u) {
            for (unsigned t = 0; t < nt; t++) tiles.push_back(TileRef{unsigned(p), t});
        } else {
            // rectangular tiles row group by row group (tile_bits), then the
            // packed tail's
            const unsigned rows = 4u * (64u / P.wx), sh = tile_bits(P);
            const unsigned groups = (unsigned(P.g.n[1]) + rows - 1u) / rows;
            if ((uint64_t(groups) << sh) > uint64_t(kTailTile))
                return bfail(GALS_EINVAL, "gals_batch: tile index of problem %d out of range", p);
            for (unsigned ty = 0; ty < groups; ty++)
                for (unsigned tx = 0; tx < P.tiles_x; tx++)
                    tiles.push_back(TileRef{unsigned(p), (ty << sh) | tx});
            for (unsigned t = P.tiles_x * groups; t < nt; t++)
                tiles.push_back(TileRef{unsigned(p), kTailTile | (t - P.tiles_x * groups)});
        }
    }
    hipError_t e = hipMalloc(&b->d_probs64, sizeof(BatchProb<double>) * pd.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_probs64, pd.data(), sizeof(BatchProb<double>) * pd.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && b->prec == GALS_F32) {
        e = hipMalloc(&b->d_probs, sizeof(BatchProb<float>) * pf.size());
        if (e == hipSuccess)
            e = hipMemcpy(b->d_probs, pf.data(), sizeof(BatchProb<float>) * pf.size(),
                          hipMemcpyHostToDevice);
    } else if (e == hipSuccess) {
        b->d_probs = b->d_probs64;
    }
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_tiles, sizeof(TileRef) * tiles.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(TileRef) * tiles.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_device(b);
        return bhip(e, "gals_batch: upload of problem descriptors");
    }
    b->ntiles = unsigned(tiles.size());
    b->dirty = false;
    return GALS_OK;
}

// Enqueue one advance on stream s (no synchronisation, capturable).
hipError_t enqueue(gals_batch *b, void *state, void *ws, double t0, double dt, int64_t steps,
                   hipStream_t s)
{
    char *w = (char *)ws;
    void *copy = w;
    void *tab = w + tab_offset(b);
    hipError_t e = launch_batch_tables(b->prec, b->d_probs64, b->nprob, b->max_entries, tab, s);
    if (e != hipSuccess) return e;
    void *bufs[2] = {state, copy};
    for (int64_t n = 0; n < steps; n++) {
        const double t = t0 + double(n) * dt;
        const double c1 = b->period > 0 ? cos(M_PI * (t + dt) / b->period) : 1.0;
        const double c2 = b->period > 0 ? cos(M_PI * t / b->period) : 1.0;
        const double c3 = b->period > 0 ? cos(M_PI * (t + 0.5 * dt) / b->period) : 1.0;
        e = launch_batch_step(b->prec, b->mixed, b->d_probs, b->d_tiles, b->ntiles, dt, c1, c2,
                              c3, tab, bufs[n & 1], bufs[(n + 1) & 1], s);
        if (e != hipSuccess) return e;
    }
    if (steps & 1)
        e = launch_batch_copy(b->prec, b->d_probs, b->d_tiles, b->ntiles, copy, state, b->blocks, s);
    return e;
}

bool overlap(const void *a, size_t na, const void *c, size_t nc)
{
    const char *pa = (const char *)a, *pc = (const char *)c;
    return pa < pc + nc && pc < pa + na;
}

struct DevGuard {
    int old = -1;
    hipError_t err = hipSuccess;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) err = hipSetDevice(dev);
    }
    ~DevGuard()
    {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

int check_advance_args(gals_batch *b, void *state, double t0, double dt, int64_t steps, void *ws,
                       size_t wsb)
{
    if (!b) return bfail(GALS_EINVAL, "gals_batch: NULL batch");
    if (!state || !ws) return bfail(GALS_EINVAL, "gals_batch: NULL state or workspace");
    for (int p = 0; p < b->nprob; p++)
        if (!b->vel_set[p]) return bfail(GALS_EINVAL, "gals_batch: no velocity for problem %d", p);
    if (!isfinite(dt) || !(dt > 0.0)) return bfail(GALS_EINVAL, "gals_batch: dt must be > 0");
    if (!isfinite(t0)) return bfail(GALS_EINVAL, "gals_batch: t0 must be finite");
    if (steps < 0) return bfail(GALS_EINVAL, "gals_batch: steps < 0");
    if (wsb < ws_bytes(b)) return bfail(GALS_EINVAL, "gals_batch: workspace too small");
    if ((uintptr_t(state) % es(b)) || (uintptr_t(ws) % 256))
        return bfail(GALS_EINVAL, "gals_batch: misaligned state or workspace");
    if (overlap(state, size_t(b->total_elems) * es(b), ws, wsb))
        return bfail(GALS_EINVAL, "gals_batch: state and workspace overlap");
    return GALS_OK;
}

}  // namespace

extern "C" {

int gals_batch_create(gals_batch **out, int64_t nprob, const int64_t *ncell, const double *lo,
                      const double *hi, int prec, int mixed_mode, int bc, int device)
{
    if (!out) return bfail(GALS_EINVAL, "gals_batch_create: out is NULL");
    *out = nullptr;
    // the table launch puts the problem index in the grid's y dimension
    if (nprob < 1 || nprob > 65535) return bfail(GALS_EINVAL, "gals_batch_create: nprob must be 1..65535");
    if (!ncell || !lo || !hi) return bfail(GALS_EINVAL, "gals_batch_create: NULL ncell/lo/hi");
    if (prec != GALS_F32 && prec != GALS_F64) return bfail(GALS_EINVAL, "gals_batch_create: precision");
    if (mixed_mode != GALS_MIXED_CENTRAL && mixed_mode != GALS_MIXED_CELL &&
        mixed_mode != GALS_MIXED_ZERO)
        return bfail(GALS_EINVAL, "gals_batch_create: mixed-derivative mode");
    if (bc != GALS_BC_NEUMANN && bc != GALS_BC_EXTRAPOLATE)
        return bfail(GALS_EINVAL, "gals_batch_create: boundary treatment");
    gals_batch *b = new (std::nothrow) gals_batch;
    if (!b) return bfail(GALS_ENOMEM, "gals_batch_create: out of host memory");
    b->nprob = int(nprob);
    b->prec = prec;
    b->mixed = mixed_mode;
    b->bc = bc;
    b->device = device;
    b->g.resize(nprob);
    b->off.resize(nprob);
    b->tab.resize(nprob);
    b->S.assign(16 * nprob, 0.0);
    b->vel_set.assign(nprob, 0);
    const int64_t esz = prec == GALS_F32 ? 4 : 8;
    int64_t offs = 0, tabs = 0;
    for (int64_t p = 0; p < nprob; p++) {
        Geom &g = b->g[p];
        memset(&g, 0, sizeof(g));
        g.dim = 2;
        g.bc = bc;
        g.n[2] = 1;
        g.h[2] = g.inv_h[2] = 1.0;
        for (int a = 0; a < 2; a++) {
            const int64_t nc = ncell[2 * p + a];
            const double l = lo[2 * p + a], h = hi[2 * p + a];
            if (nc < 2 || nc > (1 << 20) || !isfinite(l) || !isfinite(h) || !(h > l)) {
                delete b;
                return bfail(GALS_EINVAL, "gals_batch_create: problem %lld axis %d invalid",
                             (long long)p, a);
            }
            g.nc[a] = int(nc);
            g.n[a] = int(nc + 1);
            g.lo[a] = l;
            g.h[a] = (h - l) / double(nc);
            g.inv_h[a] = 1.0 / g.h[a];
            g.top[a] = node_coord(l, nc, g.h[a]);
        }
        g.nodes = int64_t(g.n[0]) * g.n[1];
        geom_finish(g);
        g.pitch = round_up(g.n[0], 64);
        g.plane = g.pitch * g.n[1];
        if (g.plane * esz >= (int64_t(1) << 31)) {
            delete b;
            return bfail(GALS_EINVAL, "gals_batch_create: problem %lld plane of 2 GiB or more",
                         (long long)p);
        }
        b->off[p] = offs;
        offs += 3 * g.plane;  // planes are multiples of 64 elements: alignment kept
        b->tab[p] = tabs;
        tabs += round_up(int64_t(g.n[0] + g.n[1]) * kJet, 64);
        const int entries = g.n[0] + g.n[1];
        if (entries > b->max_entries) b->max_entries = entries;
    }
    b->total_elems = offs;
    b->tab_elems = tabs;
    if (device >= 0) {
        int count = 0, cus = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e == hipSuccess && (device >= count)) e = hipErrorInvalidDevice;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        if (e != hipSuccess) {
            delete b;
            return bhip(e, "gals_batch_create: device query");
        }
        // the copy-back kernel's grid: 8 blocks of 256 threads per CU, a
        // multiple of the 8 XCDs (the step kernel takes one block per tile)
        b->blocks = (unsigned(cus) * 8u + 7u) / 8u * 8u;
    } else if (device != -1) {
        delete b;
        return bfail(GALS_EINVAL, "gals_batch_create: device %d", device);
    } else {
        b->blocks = 2048;
    }
    b->shape_key = shape_key(prec, mixed_mode, nprob, ncell);
    unsigned tuned[4];
    if (lookup_tuned(b->shape_key, tuned))
        for (int c = 0; c < 4; c++) b->class_wx[c] = tuned[c];
    *out = b;
    return GALS_OK;
}

int gals_batch_destroy(gals_batch *b)
{
    if (!b) return GALS_OK;
    if (b->device >= 0) {
        DevGuard dg(b->device);
        drop_graph(b);
        free_device(b);
    }
    delete b;
    return GALS_OK;
}

int gals_batch_layout(const gals_batch *b, int64_t *offset, int64_t *pitch, int64_t *plane,
                      int64_t *total_elems)
{
    if (!b) return bfail(GALS_EINVAL, "gals_batch_layout: NULL batch");
    for (int p = 0; p < b->nprob; p++) {
        if (offset) offset[p] = b->off[p];
        if (pitch) pitch[p] = b->g[p].pitch;
        if (plane) plane[p] = b->g[p].plane;
    }
    if (total_elems) *total_elems = b->total_elems;
    return GALS_OK;
}

int gals_batch_workspace_bytes(const gals_batch *b, size_t *bytes)
{
    if (!b || !bytes) return bfail(GALS_EINVAL, "gals_batch_workspace_bytes: NULL argument");
    *bytes = ws_bytes(b);
    return GALS_OK;
}

int gals_batch_set_velocity(gals_batch *b, int64_t p, int kind, const double *params,
                            int64_t nparams, double period)
{
    if (!b) return bfail(GALS_EINVAL, "gals_batch_set_velocity: NULL batch");
    if (p < 0 || p >= b->nprob) return bfail(GALS_EINVAL, "gals_batch_set_velocity: problem index");
    if (kind != GALS_VEL_STREAM_SIN)
        return bfail(GALS_ENOTSUP, "gals_batch_set_velocity: batches take GALS_VEL_STREAM_SIN fields");
    if (!params || nparams <= 0 || nparams % 3 || nparams / 3 > kMaxStreamModes)
        return bfail(GALS_EINVAL, "gals_batch_set_velocity: 3 parameters per mode, 1..64 modes");
    if (!isfinite(period) || period < 0.0)
        return bfail(GALS_EINVAL, "gals_batch_set_velocity: period must be finite and >= 0");
    if (b->period_set && period != b->period)
        return bfail(GALS_EINVAL, "gals_batch_set_velocity: all problems share one period");
    double S[16] = {0};
    for (int64_t k = 0; k < nparams / 3; k++) {
        const double a = params[3 * k], m = params[3 * k + 1], n = params[3 * k + 2];
        if (!isfinite(a)) return bfail(GALS_EINVAL, "gals_batch_set_velocity: non-finite amplitude");
        if (m != floor(m) || n != floor(n) || m < 1 || m > 4 || n < 1 || n > 4)
            return bfail(GALS_ENOTSUP, "gals_batch_set_velocity: wavenumbers must be integers in 1..4");
        S[4 * (int(m) - 1) + int(n) - 1] += a;
    }
    memcpy(&b->S[16 * p], S, sizeof(S));
    b->vel_set[p] = 1;
    b->period = period;
    b->period_set = true;
    b->dirty = true;
    return GALS_OK;
}

int gals_batch_set_tiles(gals_batch *b, const int *wave_width_per_class)
{
    if (!b || !wave_width_per_class) return bfail(GALS_EINVAL, "gals_batch_set_tiles: NULL argument");
    for (int c = 0; c < 4; c++) {
        const int w = wave_width_per_class[c];
        if (w != 64 && w != 32 && w != 16 && w != 0)
            return bfail(GALS_EINVAL, "gals_batch_set_tiles: wave width must be 64, 32, 16 or 0");
    }
    for (int c = 0; c < 4; c++) b->class_wx[c] = unsigned(wave_width_per_class[c]);
    b->dirty = true;
    return GALS_OK;
}

int gals_batch_get_tiles(const gals_batch *b, int *wave_width_per_class)
{
    if (!b || !wave_width_per_class) return bfail(GALS_EINVAL, "gals_batch_get_tiles: NULL argument");
    for (int c = 0; c < 4; c++) wave_width_per_class[c] = int(b->class_wx[c]);
    return GALS_OK;
}

int gals_batch_advance(gals_batch *b, void *state, double t0, double dt, int64_t steps,
                       int use_graph, void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = check_advance_args(b, state, t0, dt, steps, workspace, workspace_bytes);
    if (rc != GALS_OK) return rc;
    if (steps == 0) return GALS_OK;
    if (b->device < 0) return bfail(GALS_EINVAL, "gals_batch_advance: host-only batch (device -1)");
    if (use_graph && !stream)
        return bfail(GALS_EINVAL, "gals_batch_advance: graph capture needs a non-null stream");
    DevGuard dg(b->device);
    if (dg.err != hipSuccess) return bhip(dg.err, "gals_batch_advance: hipSetDevice");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bhip(e, "gals_batch_advance: pending HIP error");
    rc = upload(b);
    if (rc != GALS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        e = enqueue(b, state, workspace, t0, dt, steps, s);
        return e == hipSuccess ? GALS_OK : bhip(e, "gals_batch_advance: launch");
    }
    const bool hit = b->gexec && b->gk_state == state && b->gk_ws == workspace &&
                     b->gk_stream == stream && b->gk_t0 == t0 && b->gk_dt == dt &&
                     b->gk_steps == steps;
    if (!hit) {
        drop_graph(b);
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bhip(e, "gals_batch_advance: begin capture");
        hipError_t le = enqueue(b, state, workspace, t0, dt, steps, s);
        e = hipStreamEndCapture(s, &b->graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return bhip(e, "gals_batch_advance: graph capture");
        }
        b->gk_state = state;
        b->gk_ws = workspace;
        b->gk_stream = stream;
        b->gk_t0 = t0;
        b->gk_dt = dt;
        b->gk_steps = steps;
    }
    e = hipGraphLaunch(b->gexec, s);
    return e == hipSuccess ? GALS_OK : bhip(e, "gals_batch_advance: graph launch");
}

int gals_batch_autotune(gals_batch *b, void *state, double dt, int64_t steps, void *workspace,
                        size_t workspace_bytes, void *stream, double *best_ms)
{
    int rc = check_advance_args(b, state, 0.0, dt, steps, workspace, workspace_bytes);
    if (rc != GALS_OK) return rc;
    if (steps < 1) return bfail(GALS_EINVAL, "gals_batch_autotune: steps must be >= 1");
    if (b->device < 0) return bfail(GALS_EINVAL, "gals_batch_autotune: host-only batch");
    DevGuard dg(b->device);
    if (dg.err != hipSuccess) return bhip(dg.err, "gals_batch_autotune: hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return bhip(hipGetLastError(), "gals_batch_autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bhip(hipGetLastError(), "gals_batch_autotune: event");
    }
    bool present[4] = {false, false, false, false};
    for (int p = 0; p < b->nprob; p++) present[size_class(b->g[p].n[0])] = true;
    auto time_once = [&](float *ms) -> int {
        int r = upload(b);
        if (r != GALS_OK) return r;
        hipError_t e = enqueue(b, state, workspace, 0.0, dt, 1, s);  // warm
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = enqueue(b, state, workspace, 0.0, dt, steps, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        return e == hipSuccess ? GALS_OK : bhip(e, "gals_batch_autotune: timing");
    };
    float best = 0.0f;
    rc = time_once(&best);
    for (int c = 0; c < 4 && rc == GALS_OK; c++) {
        if (!present[c]) continue;
        const unsigned keep = b->class_wx[c];
        unsigned pick = keep;
        for (unsigned w : kShapes) {
            if (w == keep) continue;
            b->class_wx[c] = w;
            b->dirty = true;
            float ms = 0.0f;
            rc = time_once(&ms);
            if (rc != GALS_OK) break;
            if (ms < best) {
                best = ms;
                pick = w;
            }
        }
        b->class_wx[c] = pick;
        b->dirty = true;
    }
    if (rc == GALS_OK) rc = upload(b);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == GALS_OK) record_tuned(b->shape_key, b->class_wx);
    if (rc == GALS_OK && best_ms) *best_ms = double(best);
    return rc;
}

}  // extern "C"
