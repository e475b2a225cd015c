// mp_api.hip -- host driver and C ABI of libmproj (declared in include/mproj.h).
//
// Owns the multigrid hierarchy and workspace of one context, runs the V-cycle,
// the FP64 iterative refinement around FP32 V-cycles, and the projection
// phases (right-hand side, solve, velocity correction) as kernel sequences on
// the caller's stream.  The only device->host transfers are small scalar
// read-backs (norms, counts) into pinned memory.
#include "../../include/mproj.h"
#include "mp_base.h"
#include "mp_device.h"
#include "mp_kernels.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

namespace {

using mp::Dims;

constexpr int kMaxBottomCells = 16384;
constexpr int kScal = 64;  // device scalar slots
// scalar slots
// (S_BIT, the running count of bottom-solve iterations of a solve, follows
// S_RR so that one read-back per residual check takes both)
enum {
    S_MEAN = 0,
    S_NB2 = 1,
    S_RR = 2,
    S_BIT = 3,
    S_BAD = 4,
    S_GAUGE = 5,
    S_ZERO = 6,
    S_NMEAN = 7,
    S_PAIR0 = 8,
    S_DEF = 12,
    S_BINV = 13  // 1 when the bottom grid's inverse G is usable (read by the kernels)
};

struct Level {
    Dims d;
    double h;
    void* x = nullptr;   // current iterate (T)
    void* x2 = nullptr;  // second iterate buffer for out-of-place sweeps
    void* b = nullptr;   // right-hand side (T)
    void* cx = nullptr;
    void* cy = nullptr;
    void* cz = nullptr;
    bool own_x = false, own_b = false, own_c = false, own_x2 = false;
    bool fused = false;  // both colours in one launch on this level
    bool blk = false;    // register-blocked kernels (finest level, cell mode)
    bool fsw = false;    // ... with both colours of a sweep in one pass
    bool blkf = false;   // register-blocked kernels with stored face coefficients
    bool pair = false;   // both colours in one launch, one red and one black cell per thread
};

constexpr long long kCoarseCells = 4096;  // levels at or below may run in one workgroup (LDS permitting)
constexpr long long kWaveBottomCells = 256;
constexpr long long kFusedMinCells = 1LL << 22;  // fused sweeps on levels at least this large
constexpr long long kPairMaxCells = 1LL << 18;   // one-launch pair sweeps on levels at most this large

// Multigrid coarsening: halve every axis while all extents are even and
// at least 4 (the coarsest grid keeps >= 2 cells per axis).
inline bool can_coarsen(int nx, int ny, int nz)
{
    return nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx >= 4 && ny >= 4 && nz >= 4;
}

// The cell-centred hierarchy also stops at a grid small enough for the direct
// bottom solve (its inverse costs less than the coarser levels' cycles).
inline bool mac_can_coarsen(int nx, int ny, int nz)
{
    return can_coarsen(nx, ny, nz) && (long long)nx * ny * nz > mp::kDirectBottomCells;
}

// Nodal projection (Sec. 3.2 Step 11): its own node hierarchy, allocated on
// the first mp_nodal_project / mp_nodal_apply call.
struct NLevel {
    mp::NDims d;
    double h = 0.0;
    long long nn = 0;  // nodes
    void* x = nullptr;
    void* b = nullptr;
    void* r = nullptr;
    void* sig = nullptr;  // cell sigma in the V-cycle's precision
    bool own_x = false, own_b = false, own_sig = false;
    bool col = false;    // z-marching column kernels
    bool pair = false;   // two colours per pass (out of place: x2)
    void* x2 = nullptr;
};

struct NodalState {
    std::vector<NLevel> lv;
    double* b64 = nullptr;          // FP64 right-hand side on the finest nodes
    double* bottom_work = nullptr;  // 4 * coarsest nodes
    double* partials = nullptr;     // per-block partial sums of the nodal reductions
    int coarse_start = -1;          // first level of the single-workgroup coarse cycle, -1 = off
    long long sig_serial = -1;      // mapping the sigma pyramid was built from
    int nb = 1;                     // blocks of the grid-stride reductions over the finest nodes
};

constexpr long long kNodalBottomMax = 16384;  // nodes of the coarsest nodal grid

inline mp::NDims node_dims(const Dims& d)
{
    return mp::NDims{d.nx, d.ny, d.nz, d.px, d.py, d.pz, d.nx + (d.px ? 0 : 1), d.ny + (d.py ? 0 : 1),
                     d.nz + (d.pz ? 0 : 1)};
}

}  // namespace

struct mp_ctx {
    mp_config cfg;
    Dims d0;
    long long n0 = 0;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    double *c64x = nullptr, *c64y = nullptr, *c64z = nullptr;
    double *beta0 = nullptr, *ccell = nullptr, *b64 = nullptr;
    double *partials = nullptr, *dscal = nullptr, *bottom_work = nullptr;
    // b64 holds the raw right-hand side and its mean is *b_shift (subtracted
    // by the residual), or b64 is mean-zero (nullptr)
    const double* b_shift = nullptr;
    double* ginv = nullptr;  // inverse G of the bottom grid (<= kDirectBottomCells cells), or nullptr
    // G is built on a second stream (it is first needed at the end of the
    // first V-cycle's descent): ev_coef orders it after the coefficient
    // pyramid, ev_inv orders the first bottom solve after it
    hipStream_t side = nullptr;
    hipEvent_t ev_coef = nullptr, ev_inv = nullptr;
    bool inv_pending = false;
    long long npartials = 0;     // doubles in partials
    double* scanw = nullptr;     // scratch of the one-dimensional scans when partials is too small
    long long scanw_cap = 0;
    double* hscal = nullptr;  // pinned host
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t evm[2] = {nullptr, nullptr};  // around the last mapping / coefficient import
    double ms_setup = 0.0;                   // its duration
    std::vector<hipEvent_t> kev;
    std::vector<double> kev_bytes;
    int kev_used = 0;
    int nbz = 1;            // partials written by the z-marching reductions
    bool cell_mode = false;  // finest level reads cell values beta0/rho (faces formed on the fly)
    float* ccell32 = nullptr;  // FP32 half reciprocals 0.5 / c of the cell values (mixed precision)
    int coarse_start = -1;  // first level of the single-workgroup coarse cycle, -1 = off
    bool phi_aligned = true;      // the caller's iterate allows 16-byte accesses
    int geometry = -1;                  // geometry of the last successful mapping
    double* sbar = nullptr;             // lateral average of S (velocity-split source)
    long long sbar_n = 0;
    long long nm = 0;                   // radii of the irregular base state (0: odd extents)
    long long* rad_offs = nullptr;      // octant cells of radius m: rad_list[rad_offs[m] .. rad_offs[m+1])
    unsigned* rad_list = nullptr;       // built on the device at the first Average
    double* fold = nullptr;             // one value per octant cell (the eight mirror cells summed)
    double* avg_irr = nullptr;          // radius averages (the uniform Average interpolates them)
    double* seff = nullptr;             // S - Sbar on the cells (split source after a uniform spherical mapping)
    int map_n1d = 0;                    // table of the last mapping: entries, spacing, star centre
    double map_dr = 0.0;
    double map_center[3] = {0.0, 0.0, 0.0};
    double* ir_phi = nullptr;     // refinement update fused into the V-cycle's last pass
    const double* ir_s = nullptr;  // (phi += ir_s[0] * e), or nullptr
    bool ir_fresh = false;         // phi is zero before that update (written, not read)
    int extra_post = 0;            // finest-level post-smoothing sweeps beyond nu2 in this V-cycle
    bool b32_ready = false;        // the right-hand side's scaled FP32 copy and its pairs are written
    bool have_coefs = false, have_base = false;
    long long map_serial = 0;  // successful mappings so far
    NodalState* nd = nullptr;
    std::string err;
};

namespace {

int fail(mp_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(mp_ctx* c, int code, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                                            \
    do {                                                                                                             \
        hipError_t e_ = (call);                                                                                      \
        if (e_ != hipSuccess) return fail((ctx), MP_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

bool log_on() { return getenv("MP_LOG") && getenv("MP_LOG")[0] == '1'; }

// Error-path testing: MP_TEST_FAIL_ALLOC=<name> makes the named workspace
// allocation report failure (after it has been made), so that the recovery
// path runs without exhausting device memory.
bool test_fail_alloc(const char* name)
{
    const char* v = getenv("MP_TEST_FAIL_ALLOC");
    return v && strcmp(v, name) == 0;
}

template <typename T>
T* dalloc(long long n, hipError_t& e)
{
    void* p = nullptr;
    e = hipMalloc(&p, (size_t)(n > 0 ? n : 1) * sizeof(T));
    return (T*)p;
}

int check_config(const mp_config* c, mp_ctx* ctx)
{
    if (!c) return fail(ctx, MP_ERR_ARG, "config is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(ctx, MP_ERR_ARG, "grid extents must be >= 1");
    if ((long long)c->nx * c->ny * c->nz > (1LL << 34)) return fail(ctx, MP_ERR_ARG, "grid too large");
    if (!(c->h > 0.0) || !isfinite(c->h)) return fail(ctx, MP_ERR_ARG, "h must be positive");
    for (int a = 0; a < 3; a++)
        if (c->bc[a] != MP_BC_PERIODIC && c->bc[a] != MP_BC_NEUMANN) return fail(ctx, MP_ERR_ARG, "bad bc[%d]", a);
    if (c->precision != MP_FP64 && c->precision != MP_MIXED) return fail(ctx, MP_ERR_ARG, "bad precision");
    if (!(c->rtol > 0.0) || c->rtol >= 1.0) return fail(ctx, MP_ERR_ARG, "rtol must be in (0, 1)");
    if (c->max_outer < 0 || c->max_outer > 10000) return fail(ctx, MP_ERR_ARG, "bad max_outer");
    if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 + c->nu2 < 1 || c->nu1 > 16 || c->nu2 > 16)
        return fail(ctx, MP_ERR_ARG, "nu1/nu2 out of range");
    if (c->cycles_per_outer < 0 || c->cycles_per_outer > 16) return fail(ctx, MP_ERR_ARG, "bad cycles_per_outer");
    if (!(c->bottom_rtol > 0.0) || c->bottom_max_iter < 1) return fail(ctx, MP_ERR_ARG, "bad bottom settings");
    if (c->demean != 0 && c->demean != 1) return fail(ctx, MP_ERR_ARG, "demean must be 0 or 1");
    if (c->smoother != MP_SMOOTH_AUTO && c->smoother != MP_SMOOTH_PER_COLOUR && c->smoother != MP_SMOOTH_FUSED)
        return fail(ctx, MP_ERR_ARG, "bad smoother");
    if (c->coarse_cycle != 0 && c->coarse_cycle != 1) return fail(ctx, MP_ERR_ARG, "coarse_cycle must be 0 or 1");
    if (c->blocked != 0 && c->blocked != 1) return fail(ctx, MP_ERR_ARG, "blocked must be 0 or 1");
    return MP_OK;
}

void free_all(mp_ctx* c)
{
    for (auto& L : c->lv) {
        if (L.own_x) (void)hipFree(L.x);
        if (L.own_x2) (void)hipFree(L.x2);
        if (L.own_b) (void)hipFree(L.b);
        if (L.own_c) {
            (void)hipFree(L.cx);
            (void)hipFree(L.cy);
            (void)hipFree(L.cz);
        }
    }
    c->lv.clear();
    double* bufs[] = {c->c64x,     c->c64y,   c->c64z,  c->beta0,       c->ccell,
                      c->b64,      c->partials, c->dscal, c->bottom_work, c->ginv};
    for (double* p : bufs)
        if (p) (void)hipFree(p);
    if (c->ccell32) (void)hipFree(c->ccell32);
    if (c->sbar) (void)hipFree(c->sbar);
    if (c->scanw) (void)hipFree(c->scanw);
    double* radbufs[] = {(double*)c->rad_offs, (double*)c->rad_list, c->fold, c->avg_irr, c->seff};
    for (double* p : radbufs)
        if (p) (void)hipFree(p);
    if (c->hscal) (void)hipHostFree(c->hscal);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->evm)
        if (e) (void)hipEventDestroy(e);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_coef) (void)hipEventDestroy(c->ev_coef);
    if (c->ev_inv) (void)hipEventDestroy(c->ev_inv);
    for (auto& e : c->kev)
        if (e) (void)hipEventDestroy(e);
    c->kev.clear();
    if (c->nd) {
        for (auto& L : c->nd->lv) {
            if (L.own_x) (void)hipFree(L.x);
            if (L.x2) (void)hipFree(L.x2);
            if (L.own_b) (void)hipFree(L.b);
            (void)hipFree(L.r);
            if (L.own_sig) (void)hipFree(L.sig);
        }
        if (c->nd->b64) (void)hipFree(c->nd->b64);
        if (c->nd->bottom_work) (void)hipFree(c->nd->bottom_work);
        if (c->nd->partials) (void)hipFree(c->nd->partials);
        delete c->nd;
        c->nd = nullptr;
    }
}

bool mixed(const mp_ctx* c) { return c->cfg.precision == MP_MIXED; }

// FP64 finest-level coefficients (refinement residual, operator, correction).
mp::Coef<double> coef64(const mp_ctx* c)
{
    if (c->cell_mode) return mp::Coef<double>{nullptr, nullptr, nullptr, c->ccell};
    return mp::Coef<double>{c->c64x, c->c64y, c->c64z, nullptr};
}

// Coefficients of level l in the precision of the V-cycle.
template <typename T>
mp::Coef<T> level_coef(const mp_ctx* c, int l)
{
    const Level& L = c->lv[l];
    if (l == 0 && c->cell_mode) {
        if constexpr (sizeof(T) == 4) return mp::Coef<T>{nullptr, nullptr, nullptr, (const T*)c->ccell32};
        else return mp::Coef<T>{nullptr, nullptr, nullptr, (const T*)c->ccell};
    }
    return mp::Coef<T>{(const T*)L.cx, (const T*)L.cy, (const T*)L.cz, nullptr};
}

int sync_read(mp_ctx* c, int first, int count)
{
    HIPCHK(c, hipMemcpyAsync(c->hscal + first, c->dscal + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int nblk(const mp_ctx* c) { return mp::red_blocks(c->n0); }

// Irregular radial base state (Sec. 3.1): with the star centre on the node
// in the middle of the box, the centre of cell (i,j,k) lies at
// h sqrt(0.75 + 2m), m = ((2i+1-nx)^2 + (2j+1-ny)^2 + (2k+1-nz)^2 - 3) / 8.
long long radius_count(const Dims& d)
{
    if (d.nx % 2 || d.ny % 2 || d.nz % 2) return 0;
    const long long a = d.nx - 1, b = d.ny - 1, e = d.nz - 1;
    return (a * a + b * b + e * e - 3) / 8 + 1;
}

// The octant list of the lateral Average (cells of the high octant grouped
// by radius, memory order within a radius) and the folded-value buffer,
// built on the device at the first Average of a context (the grid does not
// change).  Its scratch (per-plane counters, ranks, radius counts) is freed
// afterwards.
int build_radius_list(mp_ctx* c)
{
    if (c->rad_list) return MP_OK;
    const Dims& d = c->d0;
    if (c->nm == 0) return fail(c, MP_ERR_ARG, "the irregular base state needs even extents");
    const long long noct = c->n0 / 8;
    const long long cnt_bytes = mp::oct_count_bytes(d.nx, d.ny, d.nz);
    const long long wneed = mp::scan_work_doubles(c->nm);
    void *offs = nullptr, *list = nullptr, *fold = nullptr, *cnt = nullptr, *rank = nullptr, *cntm = nullptr,
         *work = nullptr;
    bool ok = hipMalloc(&offs, sizeof(long long) * (size_t)(c->nm + 1)) == hipSuccess;
    ok = ok && hipMalloc(&list, sizeof(unsigned) * (size_t)noct) == hipSuccess;
    ok = ok && hipMalloc(&fold, sizeof(double) * (size_t)noct) == hipSuccess;
    ok = ok && hipMalloc(&cnt, (size_t)cnt_bytes) == hipSuccess;
    ok = ok && hipMalloc(&rank, sizeof(unsigned) * (size_t)noct) == hipSuccess;
    ok = ok && hipMalloc(&cntm, sizeof(double) * (size_t)c->nm) == hipSuccess;
    ok = ok && hipMalloc(&work, sizeof(double) * (size_t)wneed) == hipSuccess;
    if (test_fail_alloc("radius_list")) ok = false;
    auto release = [&](bool keep) {
        void* tmp[] = {cnt, rank, cntm, work};
        for (void* p : tmp)
            if (p) (void)hipFree(p);
        if (!keep) {
            void* res[] = {offs, list, fold};
            for (void* p : res)
                if (p) (void)hipFree(p);
        }
    };
    if (!ok) {
        release(false);
        (void)hipGetLastError();
        return fail(c, MP_ERR_NOMEM, "no device memory for the radius list");
    }
    mp::launch_radius_list(d.nx, d.ny, d.nz, c->nm, (unsigned*)cnt, (unsigned*)rank, (double*)cntm, (long long*)offs,
                           (unsigned*)list, (double*)work, c->stream);
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        release(false);
        return fail(c, MP_ERR_DEVICE, "building the radius list failed: %s", hipGetErrorString(e));
    }
    release(true);
    c->rad_offs = (long long*)offs;
    c->rad_list = (unsigned*)list;
    c->fold = (double*)fold;
    return MP_OK;
}

// Scratch of a one-dimensional scan over n values: the reduction partials
// when they hold it, else a buffer of the context grown to fit.
int scan_scratch(mp_ctx* c, long long n, double** out)
{
    const long long need = mp::scan_work_doubles(n);
    if (need <= c->npartials) {
        *out = c->partials;
        return MP_OK;
    }
    if (need > c->scanw_cap) {
        if (c->scanw) (void)hipFree(c->scanw);
        c->scanw = nullptr;
        c->scanw_cap = 0;
        if (hipMalloc((void**)&c->scanw, sizeof(double) * (size_t)need) != hipSuccess) {
            c->scanw = nullptr;
            (void)hipGetLastError();
            return fail(c, MP_ERR_NOMEM, "no device memory for the scan of %lld values", n);
        }
        c->scanw_cap = need;
    }
    *out = c->scanw;
    return MP_OK;
}

// Register-blocked kernels on level l (finest level with cell values only).
bool use_blk(const mp_ctx* c, int l) { return l == 0 && c->cell_mode && c->lv[0].blk && c->phi_aligned; }

// Register-blocked kernels on a level with stored face coefficients.
bool use_blkf(const mp_ctx* c, int l)
{
    return c->lv[l].blkf && !(l == 0 && (c->cell_mode || !c->phi_aligned));
}

// Coefficients of levels 1.. from level 0.
void build_pyramid(mp_ctx* c)
{
    for (size_t l = 1; l < c->lv.size(); l++) {
        Level& F = c->lv[l - 1];
        Level& C = c->lv[l];
        if (l == 1 && c->cell_mode) {
            if (mixed(c))
                mp::launch_coef_restrict_cells32(F.d, c->ccell32, (float*)C.cx, (float*)C.cy, (float*)C.cz, c->stream);
            else
                mp::launch_coef_restrict_cells<double>(F.d, c->ccell, (double*)C.cx, (double*)C.cy, (double*)C.cz,
                                                       c->stream);
        } else if (mixed(c)) {
            if (l == 1)
                mp::launch_coef_restrict<double, float>(F.d, c->c64x, c->c64y, c->c64z, (float*)C.cx, (float*)C.cy,
                                                        (float*)C.cz, c->stream);
            else
                mp::launch_coef_restrict<float, float>(F.d, (float*)F.cx, (float*)F.cy, (float*)F.cz, (float*)C.cx,
                                                       (float*)C.cy, (float*)C.cz, c->stream);
        } else {
            mp::launch_coef_restrict<double, double>(F.d, (double*)F.cx, (double*)F.cy, (double*)F.cz,
                                                     (double*)C.cx, (double*)C.cy, (double*)C.cz, c->stream);
        }
    }
    // inverse of the bottom grid's operator for the direct bottom solve, on
    // the second stream after the pyramid (S_BINV = 1 when usable; the bottom
    // kernels read it)
    if (c->ginv) {
        const Level& B = c->lv.back();
        (void)hipEventRecord(c->ev_coef, c->stream);
        (void)hipStreamWaitEvent(c->side, c->ev_coef, 0);
        if (mixed(c))
            mp::launch_bottom_inverse<float>(B.d, (const float*)B.cx, (const float*)B.cy, (const float*)B.cz, c->ginv,
                                             c->dscal + S_BINV, c->side);
        else
            mp::launch_bottom_inverse<double>(B.d, (const double*)B.cx, (const double*)B.cy, (const double*)B.cz,
                                              c->ginv, c->dscal + S_BINV, c->side);
        (void)hipEventRecord(c->ev_inv, c->side);
        c->inv_pending = true;
    }
}

// The main stream waits for the bottom inverse once, before its first use.
void wait_inverse(mp_ctx* c)
{
    if (c->inv_pending) {
        (void)hipStreamWaitEvent(c->stream, c->ev_inv, 0);
        c->inv_pending = false;
    }
}

// Event pool for per-launch timing of the finest-level smoother.
int make_timing_events(mp_ctx* c)
{
    if (!c->kev.empty()) return MP_OK;
    c->kev.assign(2048, nullptr);
    c->kev_bytes.assign(1024, 0.0);
    for (auto& ev : c->kev)
        if (hipEventCreate(&ev) != hipSuccess) return fail(c, MP_ERR_DEVICE, "hipEventCreate failed");
    return MP_OK;
}

void timed_begin(mp_ctx* c, bool on)
{
    if (on && c->kev_used + 1 < (int)c->kev.size()) (void)hipEventRecord(c->kev[c->kev_used], c->stream);
}

void timed_end(mp_ctx* c, bool on, double bytes)
{
    if (on && c->kev_used + 1 < (int)c->kev.size()) {
        (void)hipEventRecord(c->kev[c->kev_used + 1], c->stream);
        c->kev_bytes[c->kev_used / 2] = bytes;
        c->kev_used += 2;
    }
}

// One smoothing sweep on level l.  ec: coarse correction to add first
// (prolongation), or nullptr.  last: the final sweep of the V-cycle.
template <typename T>
void smooth(mp_ctx* c, int l, bool zero_init, const T* ec, bool last = false)
{
    Level& L = c->lv[l];
    const T h2 = (T)(L.h * L.h);
    const bool tm = c->cfg.kernel_timing && l == 0;
    const double cells = (double)L.d.n();
    const mp::Coef<T> C = level_coef<T>(c, l);
    if (use_blkf(c, l) && L.fsw) {
        // both colours in one pass, out of place: x read (not when zero) and
        // written, b and the three faces read; 1/8 word of coarse correction
        const double words = (zero_init ? 5.0 : 6.0) + (ec ? 0.125 : 0.0);
        timed_begin(c, tm);
        if constexpr (sizeof(T) == 4)
            mp::launch_fsw_blkf<T>(L.d, (const T*)L.x, (T*)L.x2, (const T*)L.b, C, h2,
                                   zero_init ? mp::FS_ZERO : ec ? mp::FS_PROLONG : mp::FS_PLAIN, ec, c->stream);
        timed_end(c, tm, words * sizeof(T) * cells);
        std::swap(L.x, L.x2);
        return;
    }
    if (use_blkf(c, l)) {
        for (int colour = 0; colour < 2; colour++) {
            const bool zi = zero_init && colour == 0;
            const int mode = zi ? mp::GS_ZERO : !ec ? mp::GS_PLAIN : colour == 0 ? mp::GS_E_ALL : mp::GS_E_OWN;
            // per colour: x in and out, b, three face words; 1/8 word of e
            const double words = (zi ? 5.0 : 6.0) + (ec ? 0.125 : 0.0);
            timed_begin(c, tm);
            mp::launch_gs_blkf<T>(L.d, (T*)L.x, (const T*)L.b, C, h2, colour, mode, ec, c->stream);
            timed_end(c, tm, words * sizeof(T) * cells);
        }
        return;
    }
    if (L.fsw && !C.cell && !use_blkf(c, l)) {
        // rows of 192 cells: the one-pass sweep on 256-cell strips
        const double words = (zero_init ? 5.0 : 6.0) + (ec ? 0.125 : 0.0);
        timed_begin(c, tm);
        if constexpr (sizeof(T) == 4)
            mp::launch_fsw_blkf<T>(L.d, (const T*)L.x, (T*)L.x2, (const T*)L.b, C, h2,
                                   zero_init ? mp::FS_ZERO : ec ? mp::FS_PROLONG : mp::FS_PLAIN, ec, c->stream);
        timed_end(c, tm, words * sizeof(T) * cells);
        std::swap(L.x, L.x2);
        return;
    }
    if (L.pair && !C.cell) {
        // words per cell: x_old (unless zero), b, 3 coefficients, x_new, 1/8
        // coarse e; the red neighbours evaluated again are read from cache
        const double words = (zero_init ? 0.0 : 1.0) + 1.0 + 3.0 + 1.0 + (ec ? 0.125 : 0.0);
        timed_begin(c, tm);
        mp::launch_rb_pair<T>(L.d, (const T*)L.x, (T*)L.x2, (const T*)L.b, C, h2,
                              zero_init ? mp::FS_ZERO : ec ? mp::FS_PROLONG : mp::FS_PLAIN, ec, c->stream);
        timed_end(c, tm, words * sizeof(T) * cells);
        std::swap(L.x, L.x2);
        return;
    }
    if (L.fused && !C.cell) {
        // words per cell: x_old (unless zero), b, 3 coefficients, x_new, 1/8 coarse e
        const double words = (zero_init ? 0.0 : 1.0) + 1.0 + 3.0 + 1.0 + (ec ? 0.125 : 0.0);
        timed_begin(c, tm);
        mp::launch_sweep<T>(L.d, (const T*)L.x, (T*)L.x2, (const T*)L.b, (const T*)L.cx, (const T*)L.cy,
                            (const T*)L.cz, h2, zero_init ? 1 : 0, ec, c->stream);
        timed_end(c, tm, words * sizeof(T) * cells);
        std::swap(L.x, L.x2);
        return;
    }
    if (use_blk(c, l) && L.fsw && sizeof(T) == 4) {
        // one pass for both colours, out of place: x read (not when zero) and
        // written, b and c read, one word each per cell; 1/8 word of coarse
        // correction after prolongation; 16 bytes per cell (phi in and out;
        // 8 when phi starts at zero) when the refinement update rides on the
        // sweep
        const bool iru = last && c->ir_phi != nullptr;
        const int mode = zero_init ? mp::FS_ZERO : ec ? mp::FS_PROLONG : mp::FS_PLAIN;
        const double bytes = ((zero_init ? 3.0 : 4.0) + (ec ? 0.125 : 0.0)) * sizeof(T) * cells +
                             (iru ? (c->ir_fresh ? 8.0 : 16.0) * cells : 0.0);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tm && c->kev_used + 1 < (int)c->kev.size()) {
            e0 = c->kev[c->kev_used];
            e1 = c->kev[c->kev_used + 1];
            c->kev_bytes[c->kev_used / 2] = bytes;
            c->kev_used += 2;
        }
        if constexpr (sizeof(T) == 4)
            mp::launch_fsw_blk<T>(L.d, (const T*)L.x, (T*)L.x2, (const T*)L.b, C.cell, h2, mode, ec,
                                  iru ? c->ir_phi : nullptr, iru ? c->ir_s : nullptr, iru && c->ir_fresh ? 1 : 0, e0,
                                  e1, c->stream);
        std::swap(L.x, L.x2);
        return;
    }
    if (use_blk(c, l)) {
        // per colour: x read (not when zero) and written, b and c read, all
        // as whole rows; 1/8 word of coarse correction after prolongation
        for (int colour = 0; colour < 2; colour++) {
            const bool zi = zero_init && colour == 0;
            const int mode = zi ? mp::GS_ZERO : !ec ? mp::GS_PLAIN : colour == 0 ? mp::GS_E_ALL : mp::GS_E_OWN;
            const bool iru = last && colour == 1 && c->ir_phi != nullptr;
            const double words = (zi ? 3.0 : 4.0) + (ec ? 0.125 : 0.0);
            // the fused refinement update adds 16 bytes per cell (phi in and out)
            const double bytes = words * sizeof(T) * cells + (iru ? 16.0 * cells : 0.0);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (tm && c->kev_used + 1 < (int)c->kev.size()) {
                e0 = c->kev[c->kev_used];
                e1 = c->kev[c->kev_used + 1];
                c->kev_bytes[c->kev_used / 2] = bytes;
                c->kev_used += 2;
            }
            mp::launch_gs_blk<T>(L.d, (T*)L.x, (const T*)L.b, C.cell, h2, colour, mode, ec,
                                 iru ? c->ir_phi : nullptr, iru ? c->ir_s : nullptr, e0, e1, c->stream);
        }
        return;
    }
    for (int colour = 0; colour < 2; colour++) {
        // per colour: x (both colours share every line; not read when zero),
        // coefficients (3 face words, or 1 cell word), b and x of one colour;
        // after a prolongation it is folded into the two passes (1/8 word of e)
        const bool zi = zero_init && colour == 0;
        const double words = (zi ? 0.0 : 1.0) + (C.cell ? 1.0 : 3.0) + 0.5 + (zi ? 1.0 : 0.5) + (ec ? 0.125 : 0.0);
        timed_begin(c, tm);
        if (ec)
            mp::launch_rbgs_e<T>(L.d, (T*)L.x, (const T*)L.b, C, h2, colour, colour == 0 ? 1 : 0, ec, c->stream);
        else
            mp::launch_rbgs<T>(L.d, (T*)L.x, (const T*)L.b, C, h2, colour, zi ? 1 : 0, c->stream);
        timed_end(c, tm, words * sizeof(T) * cells);
    }
}

template <typename T>
void coarse_cycle(mp_ctx* c, bool zero_init)
{
    mp::CoarseArgs<T> a;
    memset(&a, 0, sizeof(a));
    const int l0 = c->coarse_start;
    a.nlev = (int)c->lv.size() - l0;
    a.px = c->d0.px;
    a.py = c->d0.py;
    a.pz = c->d0.pz;
    a.nu1 = c->cfg.nu1;
    a.nu2 = c->cfg.nu2;
    a.zero_init = zero_init ? 1 : 0;
    a.bottom_rtol = c->cfg.bottom_rtol;
    a.bottom_maxit = c->cfg.bottom_max_iter;
    a.bottom_iters = c->dscal + S_BIT;
    a.bottom_inv = c->ginv;
    a.bottom_ok = c->dscal + S_BINV;
    wait_inverse(c);
    for (int q = 0; q < a.nlev; q++) {
        const Level& L = c->lv[l0 + q];
        mp::CoarseLevel<T>& C = a.lv[q];
        C.nx = L.d.nx;
        C.ny = L.d.ny;
        C.nz = L.d.nz;
        C.h2 = (T)(L.h * L.h);
        C.inv_h2 = (T)(1.0 / (L.h * L.h));
        C.h2d = L.h * L.h;
        C.x = (T*)L.x;
        C.b = (T*)L.b;
        C.cx = (const T*)L.cx;
        C.cy = (const T*)L.cy;
        C.cz = (const T*)L.cz;
    }
    mp::launch_coarse_cycle<T>(a, c->stream);
}

template <typename T>
void vcycle(mp_ctx* c, int l, bool zero_init)
{
    Level& L = c->lv[l];
    const int nlev = (int)c->lv.size();
    if (l == c->coarse_start) {
        coarse_cycle<T>(c, zero_init);
        return;
    }
    if (l == nlev - 1) {
        // directly when G is usable, else BiCGStab (each kernel reads S_BINV
        // and returns at once when the other one applies)
        const double* ok = c->ginv ? c->dscal + S_BINV : nullptr;
        if (c->ginv) {
            wait_inverse(c);
            mp::launch_bottom_direct<T>(L.d, c->ginv, ok, (const T*)L.b, (T*)L.x, L.h * L.h, c->stream);
        }
        mp::launch_bottom<T>(L.d, (const T*)L.b, (T*)L.x, (const T*)L.cx, (const T*)L.cy, (const T*)L.cz, L.h * L.h,
                             c->cfg.bottom_rtol, c->cfg.bottom_max_iter, zero_init ? 0 : 1, c->bottom_work,
                             c->dscal + S_BIT, ok, c->stream);
        return;
    }
    if (zero_init && c->cfg.nu1 == 0) (void)hipMemsetAsync(L.x, 0, sizeof(T) * L.d.n(), c->stream);
    for (int s = 0; s < c->cfg.nu1; s++) smooth<T>(c, l, zero_init && s == 0, (const T*)nullptr);
    Level& C = c->lv[l + 1];
    if (use_blk(c, l))
        mp::launch_rr_blk<T>(L.d, (const T*)L.x, (const T*)L.b, level_coef<T>(c, l).cell, (T)(1.0 / (L.h * L.h)),
                             (T*)C.b, c->stream);
    else if (use_blkf(c, l))
        mp::launch_rr_blkf<T>(L.d, (const T*)L.x, (const T*)L.b, level_coef<T>(c, l), (T)(1.0 / (L.h * L.h)),
                              (T*)C.b, c->stream);
    else
        mp::launch_resid_restrict<T>(L.d, (const T*)L.x, (const T*)L.b, level_coef<T>(c, l), (T)(1.0 / (L.h * L.h)),
                                     (T*)C.b, c->stream);
    vcycle<T>(c, l + 1, true);
    if (c->cfg.nu2 == 0) {
        mp::launch_prolong<T>(L.d, (T*)L.x, (const T*)C.x, c->stream);
        return;
    }
    const int nu2 = c->cfg.nu2 + (l == 0 ? c->extra_post : 0);
    for (int s = 0; s < nu2; s++) smooth<T>(c, l, false, s == 0 ? (const T*)C.x : (const T*)nullptr, s == nu2 - 1);
}

// V-cycles before the next residual check.  cycles_per_outer > 0 fixes the
// count; 0 predicts it from the contraction of the last step,
// rho = (rel / rel_prev)^(1 / m_prev): about log(rtol / rel) / log(rho)
// cycles, at least 1 and at most 4 (FP32 corrections gain nothing beyond).
// From a zero iterate the first step runs the most, kFirstCycles, instead of
// one measuring cycle: the first cycle contracts most (~1e-2), so 4 cycles
// end near 1e-6, still above the FP32 floor.  The mean rate of such a step
// includes that first cycle, so the prediction aims at half the tolerance:
// the MAC and nodal solves at 256^3 then reach 1e-10 in two steps instead of
// three.
// The contraction per cycle weakens as the smooth error components remain
// (on the stratified workloads ~0.03 for the second cycle, ~0.08 for the
// eighth), so the mean rate of the last step is discounted by a fifth: a
// prediction one cycle short costs a whole refinement step (an FP64 residual
// and a read-back) to run the missing cycle.
// Those two allowances make the predicted count about 0.4 cycle larger than
// what the workloads need: where the last predicted cycle would be used for
// at most kLastFraction of it, the step runs one cycle fewer and its last
// cycle one more finest-level post-smoothing sweep (*extra_post = 1), which
// buys ~0.1 cycle for a tenth of the cost.  The MAC solves at 256^3 to 512^3
// then take 4 cycles, and 2 cycles plus a sweep (end residual 5e-11 to
// 7e-11 against 1e-10), instead of 4 + 3.
constexpr int kFirstCycles = 4;
constexpr double kLastFraction = 0.45;

int cycles_this_step(const mp_ctx* c, int it, double rel, double rel_prev, int m_prev, bool from_zero,
                     int* extra_post = nullptr)
{
    if (extra_post) *extra_post = 0;
    if (c->cfg.cycles_per_outer > 0) return c->cfg.cycles_per_outer;
    if (it == 0) return from_zero ? kFirstCycles : 1;
    if (!(rel_prev > 0.0) || !(rel > 0.0)) return 1;
    const double rho = pow(rel / rel_prev, 1.0 / m_prev);
    if (!(rho > 0.0) || rho >= 0.5) return 1;
    const double need = log(0.5 * c->cfg.rtol / rel) / (0.8 * log(rho));
    int m = (int)ceil(need - 0.25);
    m = m < 1 ? 1 : m > 4 ? 4 : m;
    if (extra_post && c->cfg.nu2 >= 1 && m >= 2 && need - (m - 1) <= kLastFraction) {
        m -= 1;
        *extra_post = 1;
    }
    return m;
}

// Solve A phi = b64 (b64 mean-zero, ||b64||^2 = nb2 in hscal[S_NB2]).
int run_solve(mp_ctx* c, double* phi, int use_guess, mp_info* info)
{
    // the scaled FP32 right-hand side from the mean removal, for this solve only
    const bool b32_ready = c->b32_ready;
    c->b32_ready = false;
    const long long n = c->n0;
    const int nb = nblk(c);
    const double nb2 = c->hscal[S_NB2];
    const double inv_h2 = 1.0 / (c->cfg.h * c->cfg.h);
    if (info) info->levels = (int)c->lv.size();
    if (!isfinite(nb2)) return fail(c, MP_ERR_NONFINITE, "right-hand side is not finite");
    if (nb2 == 0.0) {
        HIPCHK(c, hipMemsetAsync(phi, 0, sizeof(double) * n, c->stream));
        if (info) info->rel_resid = 0.0;
        return MP_OK;
    }
    c->phi_aligned = ((uintptr_t)phi & 15) == 0;
    // a raw right-hand side is read through the blocked residual only
    if (c->b_shift && !use_blk(c, 0)) {
        mp::launch_sub_mean(c->b64, n, c->b_shift, c->stream);
        c->b_shift = nullptr;
    }
    const bool mx = mixed(c);
    // from a zero iterate, the first refinement update writes phi without
    // reading it where it rides on the one-pass finest-level sweep; else phi
    // is cleared first
    const bool fresh_ok = mx && use_blk(c, 0) && c->lv[0].fsw && c->cfg.nu2 >= 1;
    bool phi_set = use_guess != 0;
    if (!phi_set && !fresh_ok) {
        HIPCHK(c, hipMemsetAsync(phi, 0, sizeof(double) * n, c->stream));
        phi_set = true;
    }
    if (!mx) c->lv[0].x = phi;  // x2 stays the internal second buffer
    int status = MP_ERR_NOT_CONVERGED;
    double rel = 1.0, rel_prev = 1.0;
    double hist[64];
    int vc = 0, it = 0, m_prev = 1;
    for (it = 0;; it++) {
        const int p = it & 1;
        double* sp = c->dscal + S_PAIR0 + 2 * p;
        double* sq = c->dscal + S_PAIR0 + 2 * (1 - p);
        int nbr = 0;
        if (it == 0 && !use_guess) {
            // zero iterate: the residual is b (relative residual 1), so the
            // residual pass and its read-back are skipped (and the scaling
            // too when the mean removal wrote the scaled copy and both pairs)
            if (!b32_ready) mp::launch_scale32(n, c->b64, mx ? (float*)c->lv[0].b : nullptr, sp, sq, c->stream);
            rel = 1.0;
        } else {
            if (use_blk(c, 0))
                mp::launch_resid64_blk(c->d0, phi, c->b64, c->ccell, inv_h2, mx ? (float*)c->lv[0].b : nullptr,
                                       sp + 1, c->partials, &nbr, c->stream, c->b_shift);
            else
                mp::launch_resid64(c->d0, phi, c->b64, coef64(c), inv_h2, mx ? (float*)c->lv[0].b : nullptr, sp + 1,
                                   c->partials, &nbr, c->stream);
            mp::launch_final_sum(c->partials, nbr, c->dscal + S_RR, 1.0, sq, (double)n, c->stream);
            int st = sync_read(c, S_RR, 2);
            if (st) return st;
            rel = sqrt(c->hscal[S_RR] / nb2);
            if (info) info->bottom_iters_total = (int)c->hscal[S_BIT];
        }
        if (it < 64) {
            hist[it] = rel;
            if (info) info->resid_hist[it] = rel;
        }
        if (log_on()) fprintf(stderr, "[mproj] step %d rel_resid %.3e\n", it, rel);
        if (!isfinite(rel)) {
            status = MP_ERR_NONFINITE;
            fail(c, status, "residual became non-finite at step %d", it);
            break;
        }
        if (rel <= c->cfg.rtol) {
            status = MP_OK;
            break;
        }
        if (it >= c->cfg.max_outer) {
            fail(c, MP_ERR_NOT_CONVERGED, "not converged after %d steps (rel. residual %.3e)", it, rel);
            break;
        }
        if (it >= 6 && it < 64 && rel > 0.9 * hist[it - 6]) {
            if (info) info->flags |= 1;
            fail(c, MP_ERR_NOT_CONVERGED, "stagnated at step %d (rel. residual %.3e)", it, rel);
            break;
        }
        int extra = 0;
        const int m = cycles_this_step(c, it, rel, rel_prev, m_prev, it == 0 && !use_guess, &extra);
        rel_prev = rel;
        m_prev = m;
        if (mx) {
            // the last V-cycle of the step applies phi += s e in its final
            // smoother pass when the finest level runs blocked kernels
            const bool fuse_ir = use_blk(c, 0) && c->cfg.nu2 >= 1;
            c->ir_fresh = !phi_set;
            for (int k = 0; k < m; k++) {
                const bool lastc = k == m - 1;
                c->ir_phi = fuse_ir && lastc ? phi : nullptr;
                c->ir_s = sp;
                c->extra_post = lastc ? extra : 0;
                vcycle<float>(c, 0, k == 0);
                c->ir_phi = nullptr;
                c->extra_post = 0;
                vc++;
            }
            c->ir_fresh = false;
            phi_set = true;
            if (!fuse_ir) mp::launch_ir_update(n, phi, (const float*)c->lv[0].x, sp, c->stream);
        } else {
            for (int k = 0; k < m; k++) {
                c->extra_post = k == m - 1 ? extra : 0;
                vcycle<double>(c, 0, it == 0 && k == 0 && !use_guess);
                c->extra_post = 0;
                vc++;
                // out-of-place sweeps may leave the iterate in the second buffer
                if (c->lv[0].x != (void*)phi) {
                    HIPCHK(c,
                           hipMemcpyAsync(phi, c->lv[0].x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
                    std::swap(c->lv[0].x, c->lv[0].x2);
                }
            }
        }
    }
    // no refinement step ran (stopped before the first): phi is zero
    if (!phi_set) HIPCHK(c, hipMemsetAsync(phi, 0, sizeof(double) * n, c->stream));
    // gauge: mean(phi) = 0 (one reduction for every residual kernel, so that
    // the blocked and one-cell paths return the same bits)
    mp::launch_sum(phi, n, c->partials, nb, c->stream);
    mp::launch_final_sum(c->partials, nb, c->dscal + S_GAUGE, 1.0 / (double)n, nullptr, 0.0, c->stream);
    mp::launch_sub_mean(phi, n, c->dscal + S_GAUGE, c->stream);
    if (info) {
        info->outer_iters = it;
        info->vcycles = vc;
        info->rel_resid = rel;
    }
    return status;
}

// ---------------------------------------------------------------- nodal

// Node hierarchy: the cell grids of the MAC levels (halving while every
// extent is even and >= 4), with their nodes.  Level 0 of the FP64 path
// iterates on the caller's phi and reads the context's FP64 cell values.
int nd_setup(mp_ctx* c)
{
    if (c->nd) return MP_OK;
    NodalState* N = new NodalState();
    c->nd = N;
    const bool mx = mixed(c);
    const size_t tsz = mx ? sizeof(float) : sizeof(double);
    bool good = true;
    auto alloc = [&](size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes > 0 ? bytes : 1) != hipSuccess) {
            good = false;
            return (void*)nullptr;
        }
        return p;
    };
    Dims d = c->d0;
    double h = c->cfg.h;
    for (int l = 0;; l++) {
        NLevel L;
        L.d = node_dims(d);
        L.h = h;
        L.nn = (long long)L.d.mx * L.d.my * L.d.mz;
        if (mx || l > 0) {
            L.x = alloc(tsz * L.nn);
            L.b = alloc(tsz * L.nn);
            L.own_x = L.own_b = true;
        }
        L.r = alloc(tsz * L.nn);
        if (mx || l > 0) {
            L.sig = alloc(tsz * d.n());
            L.own_sig = true;
        }
        L.col = c->cfg.blocked && mp::nd_col_supported(L.d);
        L.pair = mx && L.col && mp::nd_pair_supported(L.d) && c->cfg.smoother != MP_SMOOTH_PER_COLOUR;
        if (L.pair) L.x2 = alloc(tsz * L.nn);
        N->lv.push_back(L);
        if (!can_coarsen(d.nx, d.ny, d.nz)) break;
        d = Dims{d.nx / 2, d.ny / 2, d.nz / 2, d.px, d.py, d.pz};
        h *= 2.0;
    }
    {
        const int np1 = mp::red_blocks(N->lv[0].nn), np2 = mp::nd_col_reduce_blocks(N->lv[0].d);
        N->partials = (double*)alloc(sizeof(double) * (np1 > np2 ? np1 : np2));
    }
    N->b64 = (double*)alloc(sizeof(double) * N->lv[0].nn);
    if (!mx) N->lv[0].b = N->b64;
    // single-workgroup coarse cycle: the trailing levels whose arrays fit LDS
    if (c->cfg.coarse_cycle) {
        const int nlev = (int)N->lv.size();
        std::vector<mp::NDims> dims;
        for (const auto& L : N->lv) dims.push_back(L.d);
        auto fits = [&](int from) {
            const long long b = mx ? mp::nd_coarse_lds_bytes<float>(dims.data() + from, nlev - from)
                                   : mp::nd_coarse_lds_bytes<double>(dims.data() + from, nlev - from);
            return nlev - from <= mp::kMaxCoarse && b <= mp::kCoarseLdsBytes;
        };
        int lc = nlev - 1;
        while (lc > 1 && fits(lc - 1)) lc--;
        N->coarse_start = (nlev >= 3 && fits(lc) && lc < nlev - 1) ? lc : -1;
    }
    N->bottom_work = (double*)alloc(sizeof(double) * 4 * N->lv.back().nn);
    N->nb = mp::red_blocks(N->lv[0].nn);
    if (!good) {
        (void)hipGetLastError();
        return fail(c, MP_ERR_NOMEM, "no device memory for the nodal hierarchy");
    }
    return MP_OK;
}

// Cell sigma of every nodal level from the mapped beta0/rho (FP64 cells).
void nd_build_sigma(mp_ctx* c)
{
    NodalState& N = *c->nd;
    if (N.sig_serial == c->map_serial) return;
    const bool mx = mixed(c);
    for (size_t l = 0; l < N.lv.size(); l++) {
        NLevel& L = N.lv[l];
        if (l == 0) {
            if (mx) mp::launch_nd_sigma<double, float>(L.d.nx, L.d.ny, L.d.nz, c->ccell, (float*)L.sig, 0, c->stream);
            else L.sig = c->ccell;
            continue;
        }
        const NLevel& F = N.lv[l - 1];
        if (l == 1)
            mx ? mp::launch_nd_sigma<double, float>(F.d.nx, F.d.ny, F.d.nz, c->ccell, (float*)L.sig, 1, c->stream)
               : mp::launch_nd_sigma<double, double>(F.d.nx, F.d.ny, F.d.nz, c->ccell, (double*)L.sig, 1, c->stream);
        else if (mx)
            mp::launch_nd_sigma<float, float>(F.d.nx, F.d.ny, F.d.nz, (const float*)F.sig, (float*)L.sig, 1,
                                              c->stream);
        else
            mp::launch_nd_sigma<double, double>(F.d.nx, F.d.ny, F.d.nz, (const double*)F.sig, (double*)L.sig, 1,
                                                c->stream);
    }
    N.sig_serial = c->map_serial;
}

// One V-cycle on nodal level l for A x = b (x as it stands on level l; the
// coarser levels start from zero).
template <typename T>
void nd_vcycle(mp_ctx* c, int l)
{
    NodalState& N = *c->nd;
    NLevel& L = N.lv[l];
    const int nlev = (int)N.lv.size();
    const double h2 = L.h * L.h;
    if (l == N.coarse_start) {
        mp::NdCoarseArgs<T> a;
        memset(&a, 0, sizeof(a));
        a.nlev = nlev - l;
        a.nu1 = c->cfg.nu1;
        a.nu2 = c->cfg.nu2;
        a.bottom_rtol = c->cfg.bottom_rtol;
        a.bottom_maxit = c->cfg.bottom_max_iter;
        const double hb = N.lv[nlev - 1].h;
        a.bottom_inv_h12 = 1.0 / (12.0 * hb * hb);
        a.bottom_iters = c->dscal + S_BIT;
        for (int q = 0; q < a.nlev; q++) {
            const NLevel& Q = N.lv[l + q];
            a.lv[q].d = Q.d;
            a.lv[q].h12 = (T)(12.0 * Q.h * Q.h);
            a.lv[q].inv_h12 = (T)(1.0 / (12.0 * Q.h * Q.h));
            a.lv[q].x = (T*)Q.x;
            a.lv[q].b = (const T*)Q.b;
            a.lv[q].sig = (const T*)Q.sig;
        }
        mp::launch_nd_coarse<T>(a, c->stream);
        return;
    }
    if (l == nlev - 1) {
        // on a one-level grid the finest iterate carries the previous steps
        mp::launch_nd_bottom<T>(L.d, (const T*)L.b, (T*)L.x, (const T*)L.sig, 1.0 / (12.0 * h2),
                                c->cfg.bottom_rtol, c->cfg.bottom_max_iter, l == 0 ? 1 : 0, N.bottom_work,
                                c->dscal + S_BIT, c->stream);
        return;
    }
    const T h12 = (T)(12.0 * h2), inv_h12 = (T)(1.0 / (12.0 * h2));
    auto gs = [&](int colour) {
        if (L.col) mp::launch_nd_gs_col<T>(L.d, (T*)L.x, (const T*)L.b, (const T*)L.sig, h12, colour, c->stream);
        else mp::launch_nd_gs<T>(L.d, (T*)L.x, (const T*)L.b, (const T*)L.sig, h12, colour, c->stream);
    };
    // a sweep as two passes of two colours (rows of one parity each), out of
    // place: the second pass reads the rows the first wrote
    auto sweep = [&](bool down) {
        if constexpr (sizeof(T) == 4) {
            if (L.pair) {
                // down: colours 0, 1 (even rows, x parity 0 first), then 2, 3;
                // up: colours 3, 2 (odd rows, x parity 1 first), then 1, 0
                const int r0 = down ? 0 : 1, lead = down ? 0 : 1;
                mp::launch_nd_pair<T>(L.d, (const T*)L.x, (const T*)L.x, (T*)L.x2, (const T*)L.b, (const T*)L.sig, h12,
                                      r0, lead, c->stream);
                mp::launch_nd_pair<T>(L.d, (const T*)L.x, (const T*)L.x2, (T*)L.x2, (const T*)L.b, (const T*)L.sig,
                                      h12, 1 - r0, lead, c->stream);
                std::swap(L.x, L.x2);
                return;
            }
        }
        if (down)
            for (int colour = 0; colour < 4; colour++) gs(colour);
        else
            for (int colour = 3; colour >= 0; colour--) gs(colour);
    };
    for (int s = 0; s < c->cfg.nu1; s++) sweep(true);
    NLevel& C = N.lv[l + 1];
    if (L.col)
        mp::launch_nd_resid_col<T>(L.d, (const T*)L.x, (const T*)L.b, (const T*)L.sig, inv_h12, (T*)L.r, c->stream);
    else
        mp::launch_nd_resid<T>(L.d, (const T*)L.x, (const T*)L.b, (const T*)L.sig, inv_h12, (T*)L.r, c->stream);
    mp::launch_nd_restrict<T>(L.d, C.d, (const T*)L.r, (T*)C.b, c->stream);
    if (l + 1 < nlev - 1 && l + 1 != N.coarse_start) (void)hipMemsetAsync(C.x, 0, sizeof(T) * C.nn, c->stream);
    nd_vcycle<T>(c, l + 1);
    mp::launch_nd_prolong<T>(L.d, C.d, (T*)L.x, (const T*)C.x, L.col ? 1 : 0, c->stream);
    const int nu2 = c->cfg.nu2 + (l == 0 ? c->extra_post : 0);
    for (int s = 0; s < nu2; s++) sweep(false);
}

// Solve A phi = N.b64 on the nodes (||b||^2 in hscal[S_NB2], its rms pair in
// the first scale pair): FP64 V-cycles on phi, or FP32 V-cycles inside FP64
// refinement.  phi is returned with zero node mean.
int nd_solve(mp_ctx* c, double* phi, int use_guess, mp_info* info)
{
    NodalState& N = *c->nd;
    NLevel& L0 = N.lv[0];
    const long long n = L0.nn;
    const double nb2 = c->hscal[S_NB2];
    const double inv_h12 = 1.0 / (12.0 * c->cfg.h * c->cfg.h);
    if (info) info->levels = (int)N.lv.size();
    if (!isfinite(nb2)) return fail(c, MP_ERR_NONFINITE, "right-hand side is not finite");
    if (nb2 == 0.0) {
        HIPCHK(c, hipMemsetAsync(phi, 0, sizeof(double) * n, c->stream));
        if (info) info->rel_resid = 0.0;
        return MP_OK;
    }
    if (!use_guess) HIPCHK(c, hipMemsetAsync(phi, 0, sizeof(double) * n, c->stream));
    const bool mx = mixed(c);
    if (!mx) L0.x = phi;
    const double* sig64 = c->ccell;
    int status = MP_ERR_NOT_CONVERGED;
    double rel = 1.0, rel_prev = 1.0;
    double hist[64];
    int vc = 0, it = 0, m_prev = 1;
    for (it = 0;; it++) {
        const int p = it & 1;
        double* sp = c->dscal + S_PAIR0 + 2 * p;
        double* sq = c->dscal + S_PAIR0 + 2 * (1 - p);
        int nbr = N.nb;
        if (it == 0 && !use_guess) {
            // zero iterate: the residual is b (relative residual 1)
            mp::launch_scale32(n, N.b64, mx ? (float*)L0.b : nullptr, sp, sq, c->stream);
            rel = 1.0;
        } else {
            if (L0.col)
                mp::launch_nd_resid64_col(L0.d, phi, N.b64, sig64, inv_h12, mx ? (float*)L0.b : nullptr, sp + 1,
                                          N.partials, &nbr, c->stream);
            else
                mp::launch_nd_resid64(L0.d, phi, N.b64, sig64, inv_h12, mx ? (float*)L0.b : nullptr, sp + 1,
                                      N.partials, N.nb, c->stream);
            mp::launch_final_sum(N.partials, nbr, c->dscal + S_RR, 1.0, sq, (double)n, c->stream);
            int st = sync_read(c, S_RR, 2);
            if (st) return st;
            rel = sqrt(c->hscal[S_RR] / nb2);
            if (info) info->bottom_iters_total = (int)c->hscal[S_BIT];
        }
        if (it < 64) {
            hist[it] = rel;
            if (info) info->resid_hist[it] = rel;
        }
        if (log_on()) fprintf(stderr, "[mproj] nodal step %d rel_resid %.3e\n", it, rel);
        if (!isfinite(rel)) {
            status = MP_ERR_NONFINITE;
            fail(c, status, "nodal residual became non-finite at step %d", it);
            break;
        }
        if (rel <= c->cfg.rtol) {
            status = MP_OK;
            break;
        }
        if (it >= c->cfg.max_outer) {
            fail(c, MP_ERR_NOT_CONVERGED, "nodal solve not converged after %d steps (rel. residual %.3e)", it, rel);
            break;
        }
        if (it >= 6 && it < 64 && rel > 0.9 * hist[it - 6]) {
            if (info) info->flags |= 1;
            fail(c, MP_ERR_NOT_CONVERGED, "nodal solve stagnated at step %d (rel. residual %.3e)", it, rel);
            break;
        }
        int extra = 0;
        const int m = cycles_this_step(c, it, rel, rel_prev, m_prev, it == 0 && !use_guess, &extra);
        rel_prev = rel;
        m_prev = m;
        if (mx) {
            HIPCHK(c, hipMemsetAsync(L0.x, 0, sizeof(float) * n, c->stream));
            for (int k = 0; k < m; k++) {
                c->extra_post = k == m - 1 ? extra : 0;
                nd_vcycle<float>(c, 0);
                c->extra_post = 0;
                vc++;
            }
            mp::launch_ir_update(n, phi, (const float*)L0.x, sp, c->stream);
        } else {
            for (int k = 0; k < m; k++) {
                c->extra_post = k == m - 1 ? extra : 0;
                nd_vcycle<double>(c, 0);
                c->extra_post = 0;
                vc++;
            }
        }
    }
    mp::launch_sum(phi, n, N.partials, N.nb, c->stream);
    mp::launch_final_sum(N.partials, N.nb, c->dscal + S_GAUGE, 1.0 / (double)n, nullptr, 0.0, c->stream);
    mp::launch_sub_mean(phi, n, c->dscal + S_GAUGE, c->stream);
    if (info) {
        info->outer_iters = it;
        info->vcycles = vc;
        info->rel_resid = rel;
    }
    return status;
}

// Duration of the mapping or coefficient import just completed (its events
// have been passed: the caller read a scalar back after the second).
void record_setup_time(mp_ctx* c)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->evm[0], c->evm[1]) == hipSuccess) c->ms_setup = ms;
}

void finish_timing(mp_ctx* c, mp_info* info)
{
    if (!info) return;
    info->ms_setup = c->ms_setup;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) info->ms_rhs = ms;
    if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) == hipSuccess) info->ms_solve = ms;
    if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) info->ms_correct = ms;
    if (c->cfg.kernel_timing) {
        double tot = 0.0, bytes = 0.0;
        int cnt = 0;
        for (int q = 0; q + 1 < c->kev_used; q += 2) {
            if (hipEventElapsedTime(&ms, c->kev[q], c->kev[q + 1]) == hipSuccess) {
                tot += ms;
                bytes += c->kev_bytes[q / 2];
                cnt++;
            }
        }
        info->smooth_ms_total = tot;
        info->smooth_launches = cnt;
        info->smooth_bytes = bytes;
    }
    info->smooth_form = c->lv[0].fsw ? 1 : 0;
}

void reset_info(mp_info* info)
{
    if (info) memset(info, 0, sizeof(*info));
}

}  // namespace

extern "C" {

const char* mp_version(void) { return "mproj 0.1 (gfx950)"; }

void mp_config_default(mp_config* cfg, int nx, int ny, int nz)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->nx = nx;
    cfg->ny = ny;
    cfg->nz = nz;
    cfg->h = nz > 0 ? 1.0 / nz : 1.0;
    cfg->bc[0] = MP_BC_PERIODIC;
    cfg->bc[1] = MP_BC_PERIODIC;
    cfg->bc[2] = MP_BC_NEUMANN;
    cfg->precision = MP_MIXED;
    cfg->rtol = 1e-10;
    cfg->max_outer = 100;
    cfg->nu1 = 2;
    cfg->nu2 = 2;
    cfg->cycles_per_outer = 0;
    cfg->bottom_rtol = 1e-8;
    cfg->bottom_max_iter = 400;
    cfg->demean = 1;
    cfg->kernel_timing = 0;
    cfg->smoother = MP_SMOOTH_AUTO;
    cfg->coarse_cycle = 1;
    cfg->blocked = 1;
    cfg->stream = nullptr;
    cfg->device = 0;
}

int mp_init(const mp_config* cfg, mp_ctx** out)
{
    if (!out) return MP_ERR_ARG;
    *out = nullptr;
    mp_ctx tmp;
    int st = check_config(cfg, &tmp);
    if (st) return st;
    // bottom size check (host only)
    {
        int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
        while (mac_can_coarsen(nx, ny, nz)) {
            nx /= 2;
            ny /= 2;
            nz /= 2;
        }
        if ((long long)nx * ny * nz > kMaxBottomCells) return MP_ERR_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MP_ERR_DEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return MP_ERR_ARG;
    if (hipSetDevice(cfg->device) != hipSuccess) return MP_ERR_DEVICE;

    mp_ctx* c = new mp_ctx();
    c->cfg = *cfg;
    c->stream = (hipStream_t)cfg->stream;
    c->d0 = Dims{cfg->nx, cfg->ny, cfg->nz, cfg->bc[0] == MP_BC_PERIODIC, cfg->bc[1] == MP_BC_PERIODIC,
                 cfg->bc[2] == MP_BC_PERIODIC};
    c->n0 = c->d0.n();
    c->nm = radius_count(c->d0);
    const bool mx = mixed(c);
    const size_t tsz = mx ? sizeof(float) : sizeof(double);
    hipError_t e = hipSuccess;
    auto ok = [&](void* p) { return p != nullptr && e == hipSuccess; };
    bool good = true;
    c->c64x = dalloc<double>(c->n0, e), good &= ok(c->c64x);
    c->c64y = dalloc<double>(c->n0, e), good &= ok(c->c64y);
    c->c64z = dalloc<double>(c->n0, e), good &= ok(c->c64z);
    c->beta0 = dalloc<double>(c->n0, e), good &= ok(c->beta0);
    c->ccell = dalloc<double>(c->n0, e), good &= ok(c->ccell);
    c->b64 = dalloc<double>(c->n0, e), good &= ok(c->b64);
    if (mx) c->ccell32 = dalloc<float>(c->n0, e), good &= ok(c->ccell32);
    c->nbz = mp::zred_blocks(c->d0);
    {
        int np = c->nbz > mp::kMaxRedBlocks ? c->nbz : mp::kMaxRedBlocks;
        if (mp::blk_supported(c->d0) && mp::blk_reduce_blocks(c->d0) > np) np = mp::blk_reduce_blocks(c->d0);
        // the blocked right-hand side writes two sets of partials (b, b^2)
        if (mp::proj_blk_supported(c->d0) && 2 * mp::proj_blk_reduce_blocks(c->d0) > np)
            np = 2 * mp::proj_blk_reduce_blocks(c->d0);
        // and so does the one-cell right-hand side (b, b^2 per z-column block)
        if (2 * c->nbz > np) np = 2 * c->nbz;
        c->partials = dalloc<double>(np, e), good &= ok(c->partials);
        c->npartials = np;
    }
    c->dscal = dalloc<double>(kScal, e), good &= ok(c->dscal);
    // levels
    Dims d = c->d0;
    double h = cfg->h;
    for (int l = 0;; l++) {
        Level L;
        L.d = d;
        L.h = h;
        if (mx || l > 0) {
            void* p = nullptr;
            e = hipMalloc(&p, tsz * d.n());
            good &= e == hipSuccess;
            L.x = p;
            L.own_x = true;
            p = nullptr;
            e = hipMalloc(&p, tsz * d.n());
            good &= e == hipSuccess;
            L.b = p;
            L.own_b = true;
        } else {
            L.b = c->b64;
        }
        if (mx || l > 0) {
            void* p[3] = {nullptr, nullptr, nullptr};
            for (int a = 0; a < 3; a++) {
                e = hipMalloc(&p[a], tsz * d.n());
                good &= e == hipSuccess;
            }
            L.cx = p[0];
            L.cy = p[1];
            L.cz = p[2];
            L.own_c = true;
        } else {
            L.cx = c->c64x;
            L.cy = c->c64y;
            L.cz = c->c64z;
        }
        c->lv.push_back(L);
        if (!mac_can_coarsen(d.nx, d.ny, d.nz)) break;
        d = Dims{d.nx / 2, d.ny / 2, d.nz / 2, d.px, d.py, d.pz};
        h *= 2.0;
    }
    c->bottom_work = dalloc<double>(9 * c->lv.back().d.n(), e), good &= ok(c->bottom_work);
    if (c->lv.back().d.n() <= mp::kDirectBottomCells)
        c->ginv = dalloc<double>(mp::kDirectBottomCells * mp::kDirectBottomCells, e), good &= ok(c->ginv);
    // single-workgroup coarse cycle: trailing levels of <= kCoarseCells cells,
    // when the bottom fits one wavefront and there is more than one level
    {
        const int nlev = (int)c->lv.size();
        c->coarse_start = -1;
        if (cfg->coarse_cycle && nlev >= 2 && c->lv.back().d.n() <= kWaveBottomCells) {
            // bytes of LDS the set of levels from..nlev-1 needs (5 arrays each)
            auto lds_bytes = [&](int from) {
                long long b = c->lv[from].d.n() * (long long)tsz;  // residual scratch
                for (int q = from; q < nlev; q++) b += 5LL * c->lv[q].d.n() * (long long)tsz;
                return b;
            };
            int lc = nlev - 1;
            while (lc > 0 && c->lv[lc - 1].d.n() <= kCoarseCells && nlev - (lc - 1) <= mp::kMaxCoarse &&
                   lds_bytes(lc - 1) <= mp::kCoarseLdsBytes)
                lc--;
            if (lc == 0) lc = 1;  // the finest level keeps its own launches (its iterate may be the caller's)
            c->coarse_start = lc;
        }
        c->lv[0].blk = cfg->blocked && nlev >= 2 && mp::blk_supported(c->d0);
        // both colours of a finest-level sweep in one pass (half the bytes of
        // two colour passes; bitwise the same), unless colour passes are asked for
        c->lv[0].fsw = c->lv[0].blk && mx && mp::fsw_supported(c->d0) && cfg->smoother != MP_SMOOTH_PER_COLOUR;
        if (c->lv[0].fsw) {
            void* p = nullptr;
            e = hipMalloc(&p, tsz * c->n0);
            good &= e == hipSuccess;
            c->lv[0].x2 = p;
            c->lv[0].own_x2 = true;
        }
        for (int l = 0; l < nlev - 1; l++) {
            Level& L = c->lv[l];
            if (c->coarse_start >= 0 && l >= c->coarse_start) break;
            // FP32 levels only: the FP64 variants need too many registers
            L.blkf = cfg->blocked && mx && mp::blk_supported(L.d);
            // both colours of a sweep in one pass where rows are 128 to 512
            // cells, or 192 between walls in x
            if (l > 0)
                L.fsw = ((L.blkf && mp::fsw_supported(L.d)) || (mx && mp::fsw_narrow_supported(L.d))) &&
                        cfg->smoother != MP_SMOOTH_PER_COLOUR;
            L.fused = !L.blkf && mp::sweep_supported(L.d) &&
                      (cfg->smoother == MP_SMOOTH_FUSED ||
                       (cfg->smoother == MP_SMOOTH_AUTO && L.d.n() >= kFusedMinCells));
            // the remaining coarser levels (below the workgroup's coarse
            // set): both colours in one launch with the red cells around each
            // black cell evaluated again, where a launch costs more than the
            // level's cells.  On larger levels, and in FP64 (a true division
            // per evaluation), the repeated evaluations cost as much as the
            // second launch: there only when asked for (MP_SMOOTH_FUSED)
            L.pair = l > 0 && !L.blkf && !L.fused && mp::rb_pair_supported(L.d) &&
                     (cfg->smoother == MP_SMOOTH_FUSED ||
                      (cfg->smoother == MP_SMOOTH_AUTO && mx && L.d.n() <= kPairMaxCells));
            if (L.fused || L.pair || (l > 0 && L.fsw)) {
                void* p = nullptr;
                e = hipMalloc(&p, tsz * L.d.n());
                good &= e == hipSuccess;
                L.x2 = p;
                L.own_x2 = true;
            }
        }
    }
    if (good && hipHostMalloc((void**)&c->hscal, sizeof(double) * kScal, hipHostMallocDefault) != hipSuccess)
        good = false;
    for (auto& ev : c->ev)
        if (good && hipEventCreate(&ev) != hipSuccess) good = false;
    for (auto& ev : c->evm)
        if (good && hipEventCreate(&ev) != hipSuccess) good = false;
    if (good && c->ginv &&
        (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&c->ev_coef, hipEventDisableTiming) != hipSuccess ||
         hipEventCreateWithFlags(&c->ev_inv, hipEventDisableTiming) != hipSuccess))
        good = false;
    if (good && cfg->kernel_timing && make_timing_events(c) != MP_OK) good = false;
    if (!good) {
        free_all(c);
        delete c;
        (void)hipGetLastError();
        return MP_ERR_NOMEM;
    }
    if (hipMemsetAsync(c->dscal, 0, sizeof(double) * kScal, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_all(c);
        delete c;
        return MP_ERR_DEVICE;
    }
    if (log_on())
        fprintf(stderr, "[mproj] init %dx%dx%d levels=%zu precision=%s\n", cfg->nx, cfg->ny, cfg->nz, c->lv.size(),
                mx ? "mixed" : "fp64");
    *out = c;
    return MP_OK;
}

int mp_free(mp_ctx* c)
{
    if (!c) return MP_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
    return MP_OK;
}

const char* mp_last_error(const mp_ctx* c) { return c ? c->err.c_str() : mp::noalloc_last_error(); }

int mp_map_base_state(mp_ctx* c, int geometry, const double* beta0_1d, int n1d, double dr, const double* center,
                      const double* rho, double* cx, double* cy, double* cz)
{
    if (!c) return MP_ERR_ARG;
    if (geometry != MP_PLANAR && geometry != MP_SPHERICAL && geometry != MP_SPHERICAL_IRREGULAR &&
        geometry != MP_SPHERICAL_QUADRATIC)
        return fail(c, MP_ERR_ARG, "bad geometry");
    if (!beta0_1d || !rho) return fail(c, MP_ERR_ARG, "beta0_1d and rho are required");
    if ((cx == nullptr) != (cy == nullptr) || (cx == nullptr) != (cz == nullptr))
        return fail(c, MP_ERR_ARG, "cx, cy, cz must be all given or all NULL");
    double c0 = 0, c1 = 0, c2 = 0;
    if (geometry == MP_PLANAR) {
        if (n1d != c->cfg.nz) return fail(c, MP_ERR_ARG, "planar table needs n1d == nz (%d != %d)", n1d, c->cfg.nz);
    } else if (geometry == MP_SPHERICAL_IRREGULAR) {
        if (c->nm == 0) return fail(c, MP_ERR_ARG, "the irregular base state needs even extents");
        if ((long long)n1d != c->nm)
            return fail(c, MP_ERR_ARG, "irregular table needs one entry per radius (%d != %lld)", n1d, c->nm);
    } else {
        if (n1d < (geometry == MP_SPHERICAL_QUADRATIC ? 3 : 2))
            return fail(c, MP_ERR_ARG, "spherical table too short (%d entries)", n1d);
        if (!(dr > 0.0) || !isfinite(dr)) return fail(c, MP_ERR_ARG, "dr must be positive");
        if (!center) return fail(c, MP_ERR_ARG, "center is required for spherical geometry");
        c0 = center[0];
        c1 = center[1];
        c2 = center[2];
        if (!isfinite(c0) || !isfinite(c1) || !isfinite(c2)) return fail(c, MP_ERR_ARG, "center must be finite");
    }
    (void)hipSetDevice(c->cfg.device);

    HIPCHK(c, hipEventRecord(c->evm[0], c->stream));
    // cell mode whenever the finest level is not also the coarsest
    c->cell_mode = c->lv.size() >= 2;
    Level& L0 = c->lv[0];
    const bool mx = mixed(c);
    mp::launch_fill(c->d0, c->cfg.h, geometry, beta0_1d, n1d, dr, c0, c1, c2, rho, c->beta0, c->ccell,
                    (mx && c->cell_mode) ? c->ccell32 : nullptr, c->partials, c->stream);
    mp::launch_final_sum(c->partials, c->nbz, c->dscal + S_BAD, 1.0, nullptr, 0.0, c->stream);
    if (!c->cell_mode)
        mp::launch_faces_from_cells(c->d0, c->ccell, c->c64x, c->c64y, c->c64z, mx ? (float*)L0.cx : nullptr,
                                    mx ? (float*)L0.cy : nullptr, mx ? (float*)L0.cz : nullptr, cx, cy, cz,
                                    c->stream);
    else if (cx)
        mp::launch_faces_from_cells(c->d0, c->ccell, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, cx, cy, cz,
                                    c->stream);
    build_pyramid(c);
    HIPCHK(c, hipEventRecord(c->evm[1], c->stream));
    int st = sync_read(c, S_BAD, 1);
    if (st) return st;
    record_setup_time(c);
    if (c->hscal[S_BAD] != 0.0) {
        c->have_base = c->have_coefs = false;
        return fail(c, MP_ERR_NONFINITE, "%.0f cells with rho <= 0, beta0 <= 0 or non-finite values",
                    c->hscal[S_BAD]);
    }
    c->have_base = c->have_coefs = true;
    c->geometry = geometry;
    c->map_n1d = n1d;
    c->map_dr = dr;
    c->map_center[0] = c0;
    c->map_center[1] = c1;
    c->map_center[2] = c2;
    c->map_serial++;
    return MP_OK;
}

int mp_set_coefs(mp_ctx* c, const double* cx, const double* cy, const double* cz)
{
    if (!c) return MP_ERR_ARG;
    if (!cx || !cy || !cz) return fail(c, MP_ERR_ARG, "cx, cy, cz are required");
    (void)hipSetDevice(c->cfg.device);

    HIPCHK(c, hipEventRecord(c->evm[0], c->stream));
    Level& L0 = c->lv[0];
    const bool mx = mixed(c);
    c->cell_mode = false;
    mp::launch_import_faces(c->d0, cx, cy, cz, c->c64x, c->c64y, c->c64z, mx ? (float*)L0.cx : nullptr,
                            mx ? (float*)L0.cy : nullptr, mx ? (float*)L0.cz : nullptr, c->partials, c->stream);
    mp::launch_final_sum(c->partials, c->nbz, c->dscal + S_BAD, 1.0, nullptr, 0.0, c->stream);
    build_pyramid(c);
    HIPCHK(c, hipEventRecord(c->evm[1], c->stream));
    int st = sync_read(c, S_BAD, 1);
    if (st) return st;
    record_setup_time(c);
    if (c->hscal[S_BAD] != 0.0) {
        c->have_coefs = false;
        return fail(c, MP_ERR_NONFINITE, "%.0f negative or non-finite face coefficients", c->hscal[S_BAD]);
    }
    c->have_coefs = true;
    return MP_OK;
}

// Prepare b64 from its raw form already in b64 (nb_sum partial sums in
// partials): mean -> S_MEAN, remove it and ||b||^2 -> S_NB2, rms -> first
// scale pair (nb: blocks of the grid-stride pass).  moments: the partials
// are followed by nb_sum partial sums of b^2, from which the mean and a scale
// (the rms of b - mean from the two moments) come in one pass, so that the
// mean removal also writes the first step's scaled FP32 right-hand side.
// keep_raw (with moments): b64 keeps the raw right-hand side and the blocked
// FP64 residual subtracts the mean as it reads it, saving the write-back.
static int finish_rhs(mp_ctx* c, int nb_sum, int nb, bool moments = false, bool keep_raw = false)
{
    const long long n = c->n0;
    c->b_shift = nullptr;
    if (moments) {
        mp::launch_final_moments(c->partials, c->partials + nb_sum, nb_sum, n, c->dscal + S_MEAN, c->dscal + S_PAIR0,
                                 c->dscal + S_PAIR0 + 2, c->stream);
        mp::launch_sub_mean_sumsq(c->b64, n, c->dscal + S_MEAN, c->partials, nb, c->stream, (float*)c->lv[0].b,
                                  c->dscal + S_PAIR0, keep_raw);
        if (keep_raw) c->b_shift = c->dscal + S_MEAN;
        mp::launch_final_sum(c->partials, nb, c->dscal + S_NB2, 1.0, nullptr, 0.0, c->stream, c->dscal + S_BIT);
        c->b32_ready = true;
    } else {
        c->b32_ready = false;
        mp::launch_final_sum(c->partials, nb_sum, c->dscal + S_MEAN, 1.0 / (double)n, nullptr, 0.0, c->stream);
        mp::launch_sub_mean_sumsq(c->b64, n, c->dscal + S_MEAN, c->partials, nb, c->stream);
        mp::launch_final_sum(c->partials, nb, c->dscal + S_NB2, 1.0, c->dscal + S_PAIR0, (double)n, c->stream,
                             c->dscal + S_BIT);
    }
    int st = sync_read(c, S_MEAN, 2);
    if (st) return st;
    if (!isfinite(c->hscal[S_MEAN]) || !isfinite(c->hscal[S_NB2]))
        return fail(c, MP_ERR_NONFINITE, "non-finite right-hand side");
    if (!c->cfg.demean) {
        const double m = c->hscal[S_MEAN], nb2 = c->hscal[S_NB2];
        if (fabs(m) * sqrt((double)n) > 1e-12 * sqrt(nb2 + (double)n * m * m))
            return fail(c, MP_ERR_SINGULAR_RHS, "right-hand side has mean %.3e (demean is off)", m);
    }
    return MP_OK;
}

// The projection of mp_mac_project / mp_mac_project_split: source S, or
// S - Sbar (sbar per plane for smode 1, per irregular radius for smode 2).
static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

static int project(mp_ctx* c, double* ux, double* uy, double* uz, const double* S, const double* sbar, int smode,
                   double* phi, int use_initial_guess, mp_info* info)
{
    c->kev_used = 0;
    const int nb = nblk(c);
    const double inv_h = 1.0 / c->cfg.h;
    // register-blocked right-hand side, correction and defect (cell-value
    // coefficients, periodic x and y, 16-byte aligned caller arrays)
    const bool pblk = c->cfg.blocked && c->cell_mode && mp::proj_blk_supported(c->d0) && aligned16(ux) &&
                      aligned16(uy) && aligned16(uz) && aligned16(S) && aligned16(phi);
    int nbs = c->nbz;
    // mixed precision: the right-hand side's second moment gives the first
    // step's scale, written with the mean removal
    const bool moments = mixed(c);
    if (pblk)
        mp::launch_rhs_blk(c->d0, inv_h, c->beta0, ux, uy, uz, S, sbar, smode, c->b64, nullptr, c->partials, &nbs,
                           c->stream, moments ? c->partials + mp::proj_blk_reduce_blocks(c->d0) : nullptr);
    else
        mp::launch_mac_rhs(c->d0, inv_h, c->beta0, ux, uy, uz, S, sbar, smode, c->b64, c->partials, c->stream,
                           moments ? c->partials + c->nbz : nullptr);
    int st = finish_rhs(c, nbs, nb, moments, moments && c->lv[0].blk);
    if (st) return st;
    if (info) {
        info->rhs_norm = sqrt(c->hscal[S_NB2]);
        info->rhs_mean = -c->hscal[S_MEAN];
    }
    HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    int solve_st = run_solve(c, phi, use_initial_guess, info);
    if (solve_st != MP_OK && solve_st != MP_ERR_NOT_CONVERGED) return solve_st;
    HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
    int nbd = c->nbz;
    if (pblk) {
        mp::launch_vc_blk(c->d0, inv_h, c->ccell, c->beta0, phi, ux, uy, uz, c->stream);
        mp::launch_rhs_blk(c->d0, inv_h, c->beta0, ux, uy, uz, S, sbar, smode, nullptr, c->dscal + S_MEAN, c->partials,
                           &nbd, c->stream);
    } else {
        mp::launch_vel_correct(c->d0, inv_h, coef64(c), c->beta0, phi, ux, uy, uz, c->stream);
        mp::launch_rhs_defect(c->d0, inv_h, c->beta0, ux, uy, uz, S, sbar, smode, c->dscal + S_MEAN, c->partials,
                              c->stream);
    }
    mp::launch_final_sum(c->partials, nbd, c->dscal + S_DEF, 1.0, nullptr, 0.0, c->stream);
    HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
    st = sync_read(c, S_DEF, 1);
    if (st) return st;
    if (info) {
        const double nb2 = c->hscal[S_NB2];
        info->div_defect = nb2 > 0.0 ? sqrt(c->hscal[S_DEF] / nb2) : sqrt(c->hscal[S_DEF]);
        finish_timing(c, info);
    }
    return solve_st;
}

static int project_checks(mp_ctx* c, double* ux, double* uy, double* uz, const double* S, double* phi)
{
    if (!ux || !uy || !uz || !S || !phi) return fail(c, MP_ERR_ARG, "ux, uy, uz, S and phi are required");
    if (!c->have_base) return fail(c, MP_ERR_STATE, "mp_map_base_state has not succeeded on this context");
    if (!c->have_coefs) return fail(c, MP_ERR_STATE, "face coefficients missing");
    return MP_OK;
}

int mp_mac_project(mp_ctx* c, double* ux, double* uy, double* uz, const double* S, double* phi,
                   int use_initial_guess, mp_info* info)
{
    if (!c) return MP_ERR_ARG;
    reset_info(info);
    int st = project_checks(c, ux, uy, uz, S, phi);
    if (st) return st;
    (void)hipSetDevice(c->cfg.device);
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    return project(c, ux, uy, uz, S, nullptr, 0, phi, use_initial_guess, info);
}

// A device buffer of the context holding at least n doubles (grown on demand).
static int ensure_buffer(mp_ctx* c, double** p, long long* cap, long long n, const char* what)
{
    if (*p && *cap >= n) return MP_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc((void**)p, sizeof(double) * (size_t)(n > 0 ? n : 1)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, MP_ERR_NOMEM, "no device memory for %s", what);
    }
    *cap = n;
    return MP_OK;
}

// The radius averages of phi into avg_irr (count: optional output).
static int radius_averages(mp_ctx* c, const double* phi, double* avg, double* count)
{
    int st = build_radius_list(c);
    if (st) return st;
    mp::launch_average(c->d0, c->nm, c->rad_offs, c->rad_list, phi, c->fold, avg, count, c->stream);
    return MP_OK;
}

// The star centre of the last spherical mapping is the node in the middle
// of the box (what the radii h sqrt(0.75 + 2m) of the Average assume).
static bool centred_on_middle_node(const mp_ctx* c)
{
    const double h = c->cfg.h;
    const double mid[3] = {0.5 * c->d0.nx * h, 0.5 * c->d0.ny * h, 0.5 * c->d0.nz * h};
    for (int a = 0; a < 3; a++)
        if (!(fabs(c->map_center[a] - mid[a]) <= 1e-9 * h)) return false;
    return c->nm > 0;
}

int mp_mac_project_split(mp_ctx* c, double* ux, double* uy, double* uz, const double* S, double* phi,
                         int use_initial_guess, double* sbar, mp_info* info)
{
    if (!c) return MP_ERR_ARG;
    reset_info(info);
    int st = project_checks(c, ux, uy, uz, S, phi);
    if (st) return st;
    const int geo = c->geometry;
    const bool uniform = geo == MP_SPHERICAL || geo == MP_SPHERICAL_QUADRATIC;
    if (uniform && !centred_on_middle_node(c))
        return fail(c, MP_ERR_STATE,
                    "the split source of a uniform spherical base state needs the star centred on the middle node of "
                    "a box with even extents");
    (void)hipSetDevice(c->cfg.device);
    const long long ns = geo == MP_PLANAR ? c->d0.nz : geo == MP_SPHERICAL_IRREGULAR ? c->nm : c->map_n1d;
    if (!sbar) {
        st = ensure_buffer(c, &c->sbar, &c->sbar_n, ns, "the lateral average");
        if (st) return st;
        sbar = c->sbar;
    }
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    if (geo == MP_PLANAR) {
        mp::launch_plane_average(c->d0, S, sbar, c->stream);
        return project(c, ux, uy, uz, S, sbar, 1, phi, use_initial_guess, info);
    }
    if (geo == MP_SPHERICAL_IRREGULAR) {
        st = radius_averages(c, S, sbar, nullptr);
        if (st) return st;
        return project(c, ux, uy, uz, S, sbar, 2, phi, use_initial_guess, info);
    }
    // uniform table: the radius averages interpolated onto it, filled back
    // onto the cells like beta0, S - Sbar formed once
    long long cap = c->avg_irr ? c->nm : 0;
    st = ensure_buffer(c, &c->avg_irr, &cap, c->nm, "the radius averages");
    if (st) return st;
    long long ncap = c->seff ? c->n0 : 0;
    st = ensure_buffer(c, &c->seff, &ncap, c->n0, "the split source");
    if (st) return st;
    st = radius_averages(c, S, c->avg_irr, nullptr);
    if (st) return st;
    mp::launch_average_uniform(c->nm, c->cfg.h, c->avg_irr, c->rad_offs, c->map_n1d, c->map_dr, sbar, c->stream);
    mp::launch_split_fill(c->d0, c->cfg.h, geo, sbar, c->map_n1d, c->map_dr, c->map_center, S, c->seff, c->stream);
    return project(c, ux, uy, uz, c->seff, nullptr, 0, phi, use_initial_guess, info);
}

int mp_solve(mp_ctx* c, const double* rhs, double* x, int use_initial_guess, mp_info* info)
{
    if (!c) return MP_ERR_ARG;
    reset_info(info);
    if (!rhs || !x) return fail(c, MP_ERR_ARG, "rhs and x are required");
    if (!c->have_coefs) return fail(c, MP_ERR_STATE, "no face coefficients (call mp_map_base_state or mp_set_coefs)");
    (void)hipSetDevice(c->cfg.device);
    c->kev_used = 0;
    const int nb = nblk(c);
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    mp::launch_neg_copy_sum(rhs, c->b64, c->n0, c->partials, nb, c->stream);
    int st = finish_rhs(c, nb, nb);
    if (st) return st;
    if (info) {
        info->rhs_norm = sqrt(c->hscal[S_NB2]);
        info->rhs_mean = -c->hscal[S_MEAN];
    }
    HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    int solve_st = run_solve(c, x, use_initial_guess, info);
    HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
    HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    finish_timing(c, info);
    return solve_st;
}

int mp_nodal_shape(const mp_ctx* c, int* mx, int* my, int* mz)
{
    if (!c || !mx || !my || !mz) return MP_ERR_ARG;
    const mp::NDims d = node_dims(c->d0);
    *mx = d.mx;
    *my = d.my;
    *mz = d.mz;
    return MP_OK;
}

static int nodal_ready(mp_ctx* c)
{
    if (!c->have_base) return fail(c, MP_ERR_STATE, "mp_map_base_state has not succeeded on this context");
    int st = nd_setup(c);
    if (st) return st;
    if (c->nd->lv.back().nn > kNodalBottomMax)
        return fail(c, MP_ERR_ARG, "coarsest nodal grid has %lld nodes (at most %lld)", c->nd->lv.back().nn,
                    kNodalBottomMax);
    nd_build_sigma(c);
    return MP_OK;
}

int mp_nodal_project(mp_ctx* c, double* ux, double* uy, double* uz, const double* S, double* phi,
                     int use_initial_guess, mp_info* info)
{
    if (!c) return MP_ERR_ARG;
    reset_info(info);
    if (!ux || !uy || !uz || !S || !phi) return fail(c, MP_ERR_ARG, "ux, uy, uz, S and phi are required");
    (void)hipSetDevice(c->cfg.device);
    int st = nodal_ready(c);
    if (st) return st;
    NodalState& N = *c->nd;
    const mp::NDims& d = N.lv[0].d;
    const long long nn = N.lv[0].nn;
    const double inv4h = 1.0 / (4.0 * c->cfg.h);
    const int nbc = nblk(c);
    c->kev_used = 0;
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    // mean of beta0 S over the cells, then b = L(beta0 S - m) - D(beta0 U)
    mp::launch_nd_src_sum(c->n0, c->beta0, S, c->partials, nbc, c->stream);
    mp::launch_final_sum(c->partials, nbc, c->dscal + S_MEAN, 1.0 / (double)c->n0, nullptr, 0.0, c->stream);
    const bool col = N.lv[0].col;
    int nbr = N.nb;
    if (col)
        mp::launch_nd_rhs_col(d, inv4h, c->beta0, ux, uy, uz, S, c->dscal + S_MEAN, N.b64, 0, N.partials, &nbr,
                              c->stream);
    else
        mp::launch_nd_rhs(d, inv4h, c->beta0, ux, uy, uz, S, c->dscal + S_MEAN, N.b64, 0, N.partials, N.nb, c->stream);
    // remove the node mean (rounding only, in exact arithmetic the sum is 0):
    // b then lies in the range of A, which is orthogonal to the constants
    mp::launch_final_sum(N.partials, nbr, c->dscal + S_NMEAN, 1.0 / (double)nn, nullptr, 0.0, c->stream);
    mp::launch_sub_mean_sumsq(N.b64, nn, c->dscal + S_NMEAN, N.partials, N.nb, c->stream);
    mp::launch_final_sum(N.partials, N.nb, c->dscal + S_NB2, 1.0, c->dscal + S_PAIR0, (double)nn, c->stream,
                         c->dscal + S_BIT);
    st = sync_read(c, S_MEAN, 2);
    if (st) return st;
    if (!isfinite(c->hscal[S_MEAN]) || !isfinite(c->hscal[S_NB2]))
        return fail(c, MP_ERR_NONFINITE, "non-finite nodal right-hand side");
    if (info) {
        info->rhs_norm = sqrt(c->hscal[S_NB2]);
        info->rhs_mean = c->hscal[S_MEAN];
    }
    HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    int solve_st = nd_solve(c, phi, use_initial_guess, info);
    if (solve_st != MP_OK && solve_st != MP_ERR_NOT_CONVERGED) return solve_st;
    HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
    mp::launch_nd_correct(d, inv4h, c->ccell, c->beta0, phi, ux, uy, uz, c->stream);
    int nbd = N.nb;
    if (col)
        mp::launch_nd_rhs_col(d, inv4h, c->beta0, ux, uy, uz, S, c->dscal + S_MEAN, nullptr, 1, N.partials, &nbd,
                              c->stream);
    else
        mp::launch_nd_rhs(d, inv4h, c->beta0, ux, uy, uz, S, c->dscal + S_MEAN, nullptr, 1, N.partials, N.nb,
                          c->stream);
    mp::launch_final_sum(N.partials, nbd, c->dscal + S_DEF, 1.0, nullptr, 0.0, c->stream);
    HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
    st = sync_read(c, S_DEF, 1);
    if (st) return st;
    if (info) {
        const double nb2 = c->hscal[S_NB2];
        info->div_defect = nb2 > 0.0 ? sqrt(c->hscal[S_DEF] / nb2) : sqrt(c->hscal[S_DEF]);
        finish_timing(c, info);
    }
    return solve_st;
}

int mp_nodal_apply(mp_ctx* c, const double* x, double* y)
{
    if (!c) return MP_ERR_ARG;
    if (!x || !y) return fail(c, MP_ERR_ARG, "x and y are required");
    (void)hipSetDevice(c->cfg.device);
    if (!c->have_base) return fail(c, MP_ERR_STATE, "mp_map_base_state has not succeeded on this context");
    const mp::NDims d = node_dims(c->d0);
    mp::launch_nd_apply64(d, x, c->ccell, 1.0 / (12.0 * c->cfg.h * c->cfg.h), y, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_nodal_pi(mp_ctx* c, const double* phi, double a, double s, double* pi)
{
    if (!c) return MP_ERR_ARG;
    if (!phi || !pi) return fail(c, MP_ERR_ARG, "phi and pi are required");
    if (phi == pi) return fail(c, MP_ERR_ARG, "phi and pi may not alias");
    if (!std::isfinite(a) || !std::isfinite(s)) return fail(c, MP_ERR_NONFINITE, "a and s must be finite");
    (void)hipSetDevice(c->cfg.device);
    const mp::NDims d = node_dims(c->d0);
    mp::launch_axpby((long long)d.mx * d.my * d.mz, a, s, phi, pi, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_base_radii(mp_ctx* c, double* rc, double* re)
{
    if (!c) return MP_ERR_ARG;
    if (!rc || !re) return fail(c, MP_ERR_ARG, "rc and re are required");
    if (c->nm == 0) return fail(c, MP_ERR_ARG, "the irregular base state needs even extents");
    (void)hipSetDevice(c->cfg.device);
    mp::launch_irregular_radii(c->nm, c->cfg.h, rc, re, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_enforce_hse(mp_ctx* c, long long n, const double* rc, const double* rho0, const double* g_edge,
                   double p0_base, double rho_cutoff, double* p0, long long* cutoff_index)
{
    if (!c) return MP_ERR_ARG;
    if (n < 1 || !rc || !rho0 || !g_edge || !p0) return fail(c, MP_ERR_ARG, "n >= 1, rc, rho0, g_edge, p0 required");
    if (!isfinite(p0_base) || isnan(rho_cutoff)) return fail(c, MP_ERR_ARG, "p0_base must be finite");
    (void)hipSetDevice(c->cfg.device);
    double* work = nullptr;
    int st0 = scan_scratch(c, n, &work);
    if (st0) return st0;
    mp::launch_enforce_hse(n, rc, rho0, g_edge, p0_base, rho_cutoff, p0, work, c->dscal + S_ZERO, nullptr,
                           c->stream);
    HIPCHK(c, hipGetLastError());
    if (cutoff_index) {
        int st = sync_read(c, S_ZERO, 1);
        if (st) return st;
        *cutoff_index = (long long)c->hscal[S_ZERO];
    }
    return MP_OK;
}

int mp_beta0_from_p0(mp_ctx* c, long long n, double rho0_centre, const double* p0, const double* gamma1,
                     double* beta0)
{
    if (!c) return MP_ERR_ARG;
    if (n < 1 || !p0 || !gamma1 || !beta0) return fail(c, MP_ERR_ARG, "n >= 1, p0, gamma1, beta0 required");
    if (!(rho0_centre > 0.0) || !isfinite(rho0_centre)) return fail(c, MP_ERR_ARG, "rho0_centre must be positive");
    (void)hipSetDevice(c->cfg.device);
    double* work = nullptr;
    int st0 = scan_scratch(c, n, &work);
    if (st0) return st0;
    mp::launch_beta0_from_p0(n, rho0_centre, p0, gamma1, beta0, work, c->dscal + S_ZERO, c->stream);
    int st = sync_read(c, S_ZERO, 1);
    if (st) return st;
    if (c->hscal[S_ZERO] != 0.0)
        return fail(c, MP_ERR_NONFINITE, "%.0f non-positive or non-finite p0 / Gamma1 entries", c->hscal[S_ZERO]);
    return MP_OK;
}

int mp_w0(mp_ctx* c, int geometry, long long n, const double* rc, const double* re, const double* beta0,
          const double* sbar, const double* psi, double* w0)
{
    if (!c) return MP_ERR_ARG;
    if (geometry != MP_PLANAR && geometry != MP_SPHERICAL && geometry != MP_SPHERICAL_IRREGULAR &&
        geometry != MP_SPHERICAL_QUADRATIC)
        return fail(c, MP_ERR_ARG, "bad geometry");
    if (n < 1 || !rc || !re || !beta0 || !sbar || !w0)
        return fail(c, MP_ERR_ARG, "n >= 1, rc, re, beta0, sbar, w0 required");
    (void)hipSetDevice(c->cfg.device);
    double* work = nullptr;
    int st0 = scan_scratch(c, n, &work);
    if (st0) return st0;
    mp::launch_w0(geometry == MP_PLANAR ? 0 : 1, n, rc, re, beta0, sbar, psi, w0, work, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_radius_count(const mp_ctx* c, long long* nm)
{
    if (!c || !nm) return MP_ERR_ARG;
    *nm = c->nm;
    return MP_OK;
}

int mp_average(mp_ctx* c, const double* phi, double* avg, double* count)
{
    if (!c) return MP_ERR_ARG;
    if (!phi || !avg) return fail(c, MP_ERR_ARG, "phi and avg are required");
    if (c->nm == 0) return fail(c, MP_ERR_ARG, "the irregular base state needs even extents");
    (void)hipSetDevice(c->cfg.device);
    int st = radius_averages(c, phi, avg, count);
    if (st) return st;
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_average_uniform(mp_ctx* c, const double* phi, int n1d, double dr, double* avg)
{
    if (!c) return MP_ERR_ARG;
    if (!phi || !avg) return fail(c, MP_ERR_ARG, "phi and avg are required");
    if (n1d < 1 || !(dr > 0.0) || !isfinite(dr)) return fail(c, MP_ERR_ARG, "n1d >= 1 and dr > 0 are required");
    if (c->nm == 0) return fail(c, MP_ERR_ARG, "the lateral average needs even extents");
    (void)hipSetDevice(c->cfg.device);
    long long cap = c->avg_irr ? c->nm : 0;
    int st = ensure_buffer(c, &c->avg_irr, &cap, c->nm, "the radius averages");
    if (st) return st;
    st = radius_averages(c, phi, c->avg_irr, nullptr);
    if (st) return st;
    mp::launch_average_uniform(c->nm, c->cfg.h, c->avg_irr, c->rad_offs, n1d, dr, avg, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_add_w0(mp_ctx* c, const double* w0, const double* re, long long ne, double* ux, double* uy, double* uz)
{
    if (!c) return MP_ERR_ARG;
    if (!w0 || !ux || !uy || !uz) return fail(c, MP_ERR_ARG, "w0, ux, uy and uz are required");
    if (!c->have_base) return fail(c, MP_ERR_STATE, "mp_map_base_state has not succeeded on this context");
    const bool planar = c->geometry == MP_PLANAR;
    if (planar) {
        if (c->d0.pz) return fail(c, MP_ERR_STATE, "w0 of a planar base state needs walls in z");
        if (ne != (long long)c->d0.nz + 1) return fail(c, MP_ERR_ARG, "planar w0 needs nz + 1 edge values");
    } else {
        if (!re || ne < 1) return fail(c, MP_ERR_ARG, "spherical w0 needs its ne >= 1 edges re");
    }
    (void)hipSetDevice(c->cfg.device);
    double center[3] = {c->map_center[0], c->map_center[1], c->map_center[2]};
    if (c->geometry == MP_SPHERICAL_IRREGULAR)
        for (int a = 0; a < 3; a++) center[a] = 0.5 * (a == 0 ? c->d0.nx : a == 1 ? c->d0.ny : c->d0.nz) * c->cfg.h;
    mp::launch_w0_faces(c->d0, planar ? 1 : 0, c->cfg.h, center, w0, re, ne, ux, uy, uz, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_set_kernel_timing(mp_ctx* c, int on)
{
    if (!c) return MP_ERR_ARG;
    if (on != 0 && on != 1) return fail(c, MP_ERR_ARG, "on must be 0 or 1");
    (void)hipSetDevice(c->cfg.device);
    if (on) {
        int st = make_timing_events(c);
        if (st) return st;
    }
    c->cfg.kernel_timing = on;
    return MP_OK;
}

int mp_apply(mp_ctx* c, const double* x, double* y)
{
    if (!c) return MP_ERR_ARG;
    if (!x || !y) return fail(c, MP_ERR_ARG, "x and y are required");
    if (!c->have_coefs) return fail(c, MP_ERR_STATE, "no face coefficients");
    (void)hipSetDevice(c->cfg.device);
    mp::launch_apply64(c->d0, x, coef64(c), 1.0 / (c->cfg.h * c->cfg.h), y, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

int mp_coef_grad(mp_ctx* c, const double* lam, const double* phi, double* gx, double* gy, double* gz)
{
    if (!c) return MP_ERR_ARG;
    if (!lam || !phi || !gx || !gy || !gz) return fail(c, MP_ERR_ARG, "lam, phi, gx, gy, gz are required");
    (void)hipSetDevice(c->cfg.device);
    mp::launch_coef_grad(c->d0, 1.0 / (c->cfg.h * c->cfg.h), lam, phi, gx, gy, gz, c->stream);
    HIPCHK(c, hipGetLastError());
    return MP_OK;
}

}  // extern "C"
