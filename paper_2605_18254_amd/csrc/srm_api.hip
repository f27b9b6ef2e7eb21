// srm_api.hip -- the C ABI of libsrm: context lifetime, Algorithm 1's sweep
// driver on the host, state I/O.  Every step of the sweep runs in the HIP
// kernels of k_bin.hip and k_migrate.hip on the context's stream; the host
// only computes the per-sweep scalars (swelling, adaptive grid) and reads
// back one small counter block per pass.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "srm_internal.hpp"

using namespace srm;

namespace {

thread_local std::string g_last_error;

srm_status fail(srm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
srm_status fail(srm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(SRM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

}  // namespace

namespace srm {
void set_last_error(const char *msg) { g_last_error = msg; }
}  // namespace srm

struct srm_ctx {
    srm_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t n = 0;
    int dim = 2;
    bool poly = false, plate = false;  // plate: zero-thickness disks or spherodisks
    int kshape = SRM_BALL;             // kernel family: SRM_BALL or SRM_PLATELET
    double tau = 0.0;                  // spherodisks: half-thickness / outer radius
    double rho_max = 1.0;
    double sum_rho_d = 0.0;  // sum of rho_i^dim (fraction)
    double s = 0.0;
    double s_stop = 0.0;  // swelling clamp: s_target, or a run's intermediate target scale
    int64_t t = 0;
    PBuf P{}, Q{}, T{};
    Scratch sc{};
    uint8_t *acc = nullptr;
    bool acc_valid = false;
    PBuf acc_buf{};          // storage order the acc codes refer to
    bool count_trials_on = false;
    unsigned long long *dtrials = nullptr;  // trial moves while profiling
    Counters *dcnt = nullptr;
    Counters *hcnt = nullptr;  // pinned
    double *dtmp = nullptr;    // 3n doubles: id-order staging
    int32_t *rowcnt = nullptr; // srm_pairs: partners per id, then row offsets
    int32_t *rowoff = nullptr;
    unsigned long long *dsum = nullptr;  // srm_pairs: 64-bit pair total
    int32_t *itmp = nullptr;   // n ints
    int32_t *ovf = nullptr;    // tiled migration: 8 overflow counts + 8 tile lists
    int32_t *failed = nullptr; // [0] count, then slots with accept code 0
    int32_t ovf_max_tiles = 0;
    int64_t ncap = 0;
    void *allocs[64];
    int nalloc = 0;

    // Optional device-time profile (hipEvents on the context's stream).
    bool prof_on = false;
    srm_profile prof{};
    std::vector<hipEvent_t> ev_free;
    struct Pending {
        int kind;  // 0 bin, 1 migrate (colour phase), 2 check, 3 main migration kernel
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;

    template <class T_>
    hipError_t alloc(T_ **ptr, size_t count)
    {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, (count > 0 ? count : 1) * sizeof(T_));
        if (e == hipSuccess) {
            allocs[nalloc++] = v;
            *ptr = (T_ *)v;
        }
        return e;
    }
    ~srm_ctx()
    {
        for (int i = 0; i < nalloc; ++i) (void)hipFree(allocs[i]);
        if (hcnt) (void)hipHostFree(hcnt);
        for (auto &p_ : pending) {
            (void)hipEventDestroy(p_.a);
            (void)hipEventDestroy(p_.b);
        }
        for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    }
    hipEvent_t event()
    {
        if (!ev_free.empty()) {
            hipEvent_t e = ev_free.back();
            ev_free.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Record an event on the stream (profiling only); null when off.
    hipEvent_t mark()
    {
        if (!prof_on) return nullptr;
        hipEvent_t e = event();
        if (e && hipEventRecord(e, stream) != hipSuccess) {
            ev_free.push_back(e);
            return nullptr;
        }
        return e;
    }
    void span(int kind, hipEvent_t a, hipEvent_t b)
    {
        if (a && b) pending.push_back({kind, a, b});
    }
    // After a stream synchronisation: fold completed spans into prof.
    void resolve()
    {
        for (auto &p_ : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p_.a, p_.b) == hipSuccess) {
                if (p_.kind == 0) prof.ms_bin += ms;
                else if (p_.kind == 1) prof.ms_migrate += ms;
                else if (p_.kind == 3) prof.ms_migrate_main += ms;
                else prof.ms_check += ms;
            }
            release(p_.a);
            release(p_.b);
        }
        pending.clear();
    }
    void release(hipEvent_t e)
    {
        if (e) ev_free.push_back(e);
    }
};

namespace {

int64_t cell_cap(int dim, int64_t n) { return even_cap(dim, n); }

Grid make_grid(const srm_ctx *c, double rmax)
{
    return sweep_grid(c->dim, c->p.box, c->ncap, c->p.c_m, rmax);
}

// Volume per cubed radius scale of one particle with shape radius 1: ball
// omega_d; thin platelet pi a^2 t with t = thick_ratio 2a (cylinder);
// spherodisk 2 pi A^2 h + pi^2 A h^2 + 4/3 pi h^3 (core radius A = 1 - h,
// half-thickness h = thick_ratio; Steiner's formula).
double volume_coeff(const srm_ctx *c)
{
    if (c->p.shape == SRM_SPHERODISK) {
        const double h = c->p.thick_ratio, A = 1.0 - h;
        return 2.0 * M_PI * A * A * h + M_PI * M_PI * A * h * h + 4.0 / 3.0 * M_PI * h * h * h;
    }
    if (c->plate) return 2.0 * M_PI * c->p.thick_ratio;  // pi a^2 (thick_ratio 2a)
    return (c->dim == 2) ? M_PI : 4.0 * M_PI / 3.0;
}

double fraction_at(const srm_ctx *c, double s)
{
    double vbox = 1.0;
    for (int a = 0; a < c->dim; ++a) vbox *= c->p.box[a];
    double sd = 1.0;
    for (int a = 0; a < c->dim; ++a) sd *= s;
    return volume_coeff(c) * sd * c->sum_rho_d / vbox;
}

// Sec. 2 step a: s' = min(s + c_w * s_target, clamp), the clamp being
// s_target except inside srm_run_to_fraction with an intermediate target.
double swell(const srm_ctx *c, double s)
{
    const double s1 = s + c->p.c_w * c->p.s_target;
    return (s1 < c->s_stop) ? s1 : c->s_stop;
}

// Radius scale at which the volume fraction equals f (the inverse of
// fraction_at, to rounding).
double scale_for_fraction(const srm_ctx *c, double f)
{
    double vbox = 1.0;
    for (int a = 0; a < c->dim; ++a) vbox *= c->p.box[a];
    const double sd = f * vbox / (volume_coeff(c) * c->sum_rho_d);
    return (c->dim == 2) ? sqrt(sd) : cbrt(sd);
}

hipError_t alloc_buf(srm_ctx *c, PBuf &b)
{
    hipError_t e;
    for (int a = 0; a < c->dim; ++a)
        if ((e = c->alloc(&b.x[a], c->n)) != hipSuccess) return e;
    if ((e = c->alloc(&b.id, c->n)) != hipSuccess) return e;
    if (c->poly && (e = c->alloc(&b.rho, c->n)) != hipSuccess) return e;
    if (c->plate)
        for (int a = 0; a < 3; ++a)
            if ((e = c->alloc(&b.nrm[a], c->n)) != hipSuccess) return e;
    return hipSuccess;
}

srm_status bin(srm_ctx *c, const PBuf &src, const PBuf &dst, const Grid &g)
{
    hipEvent_t e0 = c->mark();
    HIP_TRY(bin_particles(c->dim, src, dst, c->n, g, c->sc, c->dcnt, c->stream));
    c->span(0, e0, c->mark());
    if (c->prof_on) c->prof.bins += 1;
    return SRM_OK;
}

PassArgs pass_args(srm_ctx *c, const PBuf &b, const Grid &g, double s, int kind, int k)
{
    PassArgs a{};
    a.buf = b;
    a.start = c->sc.start;
    a.acc = c->acc;
    a.g = g;
    a.n = c->n;
    a.s = s;
    const double sig = s + s;
    a.sig2_mono = sig * sig;
    a.draw.key0 = (uint32_t)c->p.seed;
    a.draw.key1 = (uint32_t)(c->p.seed >> 32);
    a.draw.t = (uint32_t)c->t;
    a.draw.word = counter_word((uint32_t)kind, (uint32_t)k, 0);
    a.n_l = c->p.n_l;
    a.c_m = c->p.c_m;
    a.c_n = c->p.c_n;
    a.tau = (c->p.shape == SRM_SPHERODISK) ? c->p.thick_ratio : 0.0;
    a.ovf = c->ovf;
    a.ovf_max_tiles = c->ovf_max_tiles;
    a.failed = c->failed;
    return a;
}

// One migration pass on b (already binned with g), then the reduced global
// check; returns the overlap flag and failure count through *ov / *nfail.
srm_status run_pass(srm_ctx *c, const PBuf &b, const Grid &g, double s, int kind, int k,
                    bool want_check, int32_t *ov, int64_t *nfail)
{
    const PassArgs a = pass_args(c, b, g, s, kind, k);
    HIP_TRY(launch_fill_i32(c->ovf, 8, 0, c->stream));
    HIP_TRY(launch_fill_i32(c->failed, 1, 0, c->stream));
    hipEvent_t e0 = c->mark();
    for (int colour = 0; colour < (1 << c->dim); ++colour) {
        bool launched = false;
        int which = 0;
        // m0 .. m1 brackets the colour phase's main kernel alone
        hipEvent_t m0 = c->mark();
        hipEvent_t m1 = c->prof_on ? c->event() : nullptr;
        HIP_TRY(migrate_colour(c->dim, c->kshape, c->poly, a, colour, c->stream, &launched, m1,
                               &which));
        if (launched) {
            hipEvent_t e1 = c->mark();
            c->span(1, e0, e1);
            c->span(3, m0, m1);
            e0 = e1 ? c->mark() : nullptr;
            if (c->prof_on) {
                c->prof.launches_migrate += 1;
                c->prof.main_kernels |= which;
            }
        } else {
            c->release(m0);
            c->release(m1);
        }
    }
    if (e0) c->release(e0);
    if (c->prof_on) c->prof.passes += 1;
    if (c->count_trials_on) HIP_TRY(count_trials(c->acc, c->n, c->p.n_l, c->dtrials, c->stream));
    c->acc_valid = true;
    c->acc_buf = b;
    if (!want_check) return SRM_OK;
    HIP_TRY(launch_zero_counters(c->dcnt, c->stream));
    hipEvent_t e2 = c->mark();
    HIP_TRY(check_overlaps(c->dim, c->kshape, c->poly, a, false, c->dcnt, c->stream));
    c->span(2, e2, c->mark());
    if (c->prof_on) c->prof.checks += 1;
    HIP_TRY(hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&c->hcnt->nfail_list, c->failed, sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->resolve();
    if (ov) *ov = c->hcnt->overlap;
    if (nfail) *nfail = c->hcnt->nfail_list;
    return SRM_OK;
}

srm_status check_params(const srm_params *p)
{
    if (!p) return fail(SRM_EINVAL, "params is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(SRM_EINVAL, "dim must be 2 or 3");
    if (p->shape != SRM_BALL && p->shape != SRM_PLATELET && p->shape != SRM_SPHERODISK)
        return fail(SRM_EINVAL, "bad shape");
    if (p->shape != SRM_BALL && p->dim != 3) return fail(SRM_EINVAL, "platelets are 3D");
    if (p->shape == SRM_SPHERODISK && !(p->thick_ratio > 0.0 && p->thick_ratio < 0.5))
        return fail(SRM_EINVAL, "spherodisks need 0 < thick_ratio < 0.5");
    if (p->n < 1 || p->n > 0x7fffffffLL) return fail(SRM_EINVAL, "n out of range");
    for (int a = 0; a < p->dim; ++a)
        if (!(p->box[a] > 0.0) || !isfinite(p->box[a])) return fail(SRM_EINVAL, "box edge <= 0");
    if (!(p->s_target >= 0.0) || !isfinite(p->s_target)) return fail(SRM_EINVAL, "bad s_target");
    if (!(p->c_w >= 0.0) || !(p->c_m >= 0.0) || !(p->c_n >= 0.0) || !isfinite(p->c_m) ||
        !isfinite(p->c_w) || !isfinite(p->c_n))
        return fail(SRM_EINVAL, "rates must be finite and >= 0");
    if (p->n_k < 0 || p->n_k > 32767) return fail(SRM_EINVAL, "n_k out of range");
    if (p->n_l < 0 || p->n_l > 255) return fail(SRM_EINVAL, "n_l out of range");
    return SRM_OK;
}

}  // namespace

extern "C" {

const char *srm_last_error(void) { return g_last_error.c_str(); }

srm_status srm_init(const srm_params *p, const double *pos, const double *rho,
                    const double *normals, double s0, int64_t sweep0, int32_t mem_kind,
                    void *stream, srm_ctx **out)
{
    srm_status st = check_params(p);
    if (st) return st;
    if (!pos || !out) return fail(SRM_EINVAL, "pos and out must not be NULL");
    if (mem_kind != SRM_MEM_HOST && mem_kind != SRM_MEM_DEVICE)
        return fail(SRM_EINVAL, "bad mem_kind");
    if (p->shape != SRM_BALL && !normals) return fail(SRM_EINVAL, "platelets need normals");
    if (!(s0 >= 0.0) || !isfinite(s0)) return fail(SRM_EINVAL, "bad s0");
    if (sweep0 < 0 || sweep0 > 0xffffffffLL) return fail(SRM_EINVAL, "sweep0 out of range");

    srm_ctx *c = new (std::nothrow) srm_ctx();
    if (!c) return fail(SRM_ENOMEM, "host allocation failed");
    c->p = *p;
    if (c->p.dim == 2) c->p.box[2] = 1.0;
    c->n = (int32_t)p->n;
    c->dim = p->dim;
    c->plate = p->shape != SRM_BALL;
    c->kshape = c->plate ? SRM_PLATELET : SRM_BALL;
    c->tau = (p->shape == SRM_SPHERODISK) ? p->thick_ratio : 0.0;
    c->poly = rho != nullptr;
    c->s = s0;
    c->s_stop = p->s_target;
    c->t = sweep0;
    c->stream = (hipStream_t)stream;
    c->ncap = cell_cap(c->dim, c->n);
    auto bail = [&](srm_status s_) { delete c; return s_; };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(SRM_EDEVICE, "no HIP device"));

    const size_t n = (size_t)c->n;
    hipError_t e = hipSuccess;
    if ((e = alloc_buf(c, c->P)) || (e = alloc_buf(c, c->Q)) || (e = alloc_buf(c, c->T)) ||
        (e = c->alloc(&c->sc.cell, n)) || (e = c->alloc(&c->sc.slot, n)) ||
        (e = c->alloc(&c->sc.tmpid, n)) ||
        (e = c->alloc(&c->acc, n)) || (e = c->alloc(&c->dtmp, 3 * n)) ||
        (e = c->alloc(&c->itmp, n)) || (e = c->alloc(&c->dcnt, 1)) ||
        (e = c->alloc(&c->dtrials, 1)))
        return bail(fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    {
        // tiles per colour phase are at most prod_a ceil((ncap / 2) / T)
        const int64_t tsz = (c->dim == 3) ? 4 : 8;
        int64_t per = (c->ncap / 2 + tsz - 1) / tsz;
        if (per < 1) per = 1;
        int64_t mt = 1;
        for (int a = 0; a < c->dim; ++a) mt *= per;
        c->ovf_max_tiles = (int32_t)mt;
        if ((e = c->alloc(&c->ovf, (size_t)(8 + 8 * mt))))
            return bail(fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    }
    if ((e = c->alloc(&c->failed, n + 1)))
        return bail(fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    c->sc.cap = (int64_t)n + 2;
    if ((e = c->alloc(&c->sc.counts, (size_t)c->sc.cap)) ||
        (e = c->alloc(&c->sc.start, (size_t)c->sc.cap + 1)) ||
        (e = c->alloc(&c->sc.partials, (size_t)(c->sc.cap / 2048 + 2))))
        return bail(fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if (hipHostMalloc((void **)&c->hcnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess)
        return bail(fail(SRM_ENOMEM, "pinned allocation failed"));

    // Upload in id order into T, then bin into P (committed state).
    const hipMemcpyKind kind = (mem_kind == SRM_MEM_HOST) ? hipMemcpyHostToDevice
                                                          : hipMemcpyDeviceToDevice;
    for (int a = 0; a < c->dim; ++a)
        if (hipMemcpyAsync(c->T.x[a], pos + (size_t)a * n, n * sizeof(double), kind, c->stream))
            return bail(fail(SRM_EDEVICE, "position upload failed"));
    if (c->poly && hipMemcpyAsync(c->T.rho, rho, n * sizeof(double), kind, c->stream))
        return bail(fail(SRM_EDEVICE, "rho upload failed"));
    if (c->plate)
        for (int a = 0; a < 3; ++a)
            if (hipMemcpyAsync(c->T.nrm[a], normals + (size_t)a * n, n * sizeof(double), kind,
                               c->stream))
                return bail(fail(SRM_EDEVICE, "normal upload failed"));
    if (launch_iota(c->T.id, c->n, c->stream) != hipSuccess)
        return bail(fail(SRM_EDEVICE, "id init failed"));

    // rho_max and sum rho^dim on the host (order: ascending id).
    if (c->poly) {
        double *h = (double *)malloc(n * sizeof(double));
        if (!h) return bail(fail(SRM_ENOMEM, "host allocation failed"));
        if (hipMemcpyAsync(h, c->T.rho, n * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
            hipStreamSynchronize(c->stream)) {
            free(h);
            return bail(fail(SRM_EDEVICE, "rho readback failed"));
        }
        double m = 0.0, sd = 0.0;
        bool ok = true;
        for (size_t i = 0; i < n; ++i) {
            if (!(h[i] > 0.0) || !isfinite(h[i])) ok = false;
            if (h[i] > m) m = h[i];
            double v = 1.0;
            for (int a = 0; a < c->dim; ++a) v *= h[i];
            sd += v;
        }
        free(h);
        if (!ok) return bail(fail(SRM_EINVAL, "rho must be finite and > 0"));
        c->rho_max = m;
        c->sum_rho_d = sd;
    } else {
        c->rho_max = 1.0;
        c->sum_rho_d = (double)c->n;
    }

    // Validation: every coordinate in [0, L) (recorded by the binning
    // kernel), then no overlapping pair at s0.
    const Grid g = make_grid(c, c->s * c->rho_max);
    if (launch_zero_counters(c->dcnt, c->stream) != hipSuccess)
        return bail(fail(SRM_EDEVICE, "counter init failed"));
    if ((st = bin(c, c->T, c->P, g))) return bail(st);
    if (hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return bail(fail(SRM_EDEVICE, "initial binning failed"));
    if (c->hcnt->bad) return bail(fail(SRM_EINVAL, "a coordinate is outside [0, L) or NaN"));
    PassArgs a = pass_args(c, c->P, g, c->s, 0, 0);
    if (check_overlaps(c->dim, c->kshape, c->poly, a, true, c->dcnt, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return bail(fail(SRM_EDEVICE, "initial check failed"));
    if (c->hcnt->overlap) return bail(fail(SRM_EOVERLAP, "initial configuration overlaps at s0"));
    *out = c;
    return SRM_OK;
}

srm_status srm_free(srm_ctx *c)
{
    if (!c) return SRM_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete c;
    return SRM_OK;
}

srm_status srm_sweep(srm_ctx *c, srm_sweep_info *info)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    if (c->t >= 0xffffffffLL) return fail(SRM_EINVAL, "sweep counter exhausted (2^32 - 1)");
    const double s1 = swell(c, c->s);
    const Grid g = make_grid(c, s1 * c->rho_max);
    srm_status st;
    // Q = P, binned for the new grid.
    if ((st = bin(c, c->P, c->Q, g))) return st;
    bool committed = false;
    int32_t passes_main = 0, passes_shake = 0;
    int64_t nfail = 0;
    for (int32_t k = 1; k <= c->p.n_k; ++k) {
        if (k > 1) {
            if ((st = bin(c, c->Q, c->T, g))) return st;
            std::swap(c->Q, c->T);
        }
        int32_t ov = 1;
        if ((st = run_pass(c, c->Q, g, s1, SRM_PASS_MAIN, k, true, &ov, &nfail))) return st;
        ++passes_main;
        if (!ov) {
            committed = true;
            break;
        }
    }
    if (committed) {
        std::swap(c->P, c->Q);
        c->s = s1;
    } else {
        for (int32_t j = 1; j <= c->p.n_k; ++j) {
            if ((st = bin(c, c->P, c->T, g))) return st;
            std::swap(c->P, c->T);
            if ((st = run_pass(c, c->P, g, c->s, SRM_PASS_SHAKE, j, false, nullptr, nullptr)))
                return st;
            ++passes_shake;
        }
        if (passes_shake > 0) HIP_TRY(hipStreamSynchronize(c->stream));
        c->resolve();
    }
    c->t += 1;
    if (info) {
        info->committed = committed ? 1 : 0;
        info->passes_main = passes_main;
        info->passes_shake = passes_shake;
        for (int a = 0; a < 3; ++a) info->grid[a] = g.na[a];
        info->sweep = c->t;
        info->s = c->s;
        info->fraction = fraction_at(c, c->s);
        info->n_failed_last = nfail;
    }
    return SRM_OK;
}

srm_status srm_run_to_fraction(srm_ctx *c, double f_target, int32_t max_sweeps,
                               srm_run_info *info)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    if (max_sweeps < 0) return fail(SRM_EINVAL, "max_sweeps < 0");
    if (isnan(f_target)) return fail(SRM_EINVAL, "f_target is NaN");
    double stop = c->p.s_target;
    if (f_target > 0.0) {
        const double sf = scale_for_fraction(c, f_target);
        if (sf < stop) stop = sf;
    }
    int64_t sweeps = 0, passes = 0, shakes = 0;
    srm_status st = SRM_OK;
    c->s_stop = stop;
    while (c->s < stop) {
        if (sweeps >= max_sweeps) {
            st = fail(SRM_ENOTCONV, "no convergence in %d sweeps", max_sweeps);
            break;
        }
        srm_sweep_info si;
        srm_status e = srm_sweep(c, &si);
        if (e) {
            c->s_stop = c->p.s_target;
            return e;
        }
        ++sweeps;
        passes += si.passes_main + si.passes_shake;
        shakes += si.committed ? 0 : 1;
    }
    c->s_stop = c->p.s_target;
    if (info) {
        info->sweeps = sweeps;
        info->passes = passes;
        info->shakes = shakes;
        info->updates = passes * (int64_t)c->n;
        info->s = c->s;
        info->fraction = fraction_at(c, c->s);
    }
    return st;
}

srm_status srm_get_state(srm_ctx *c, double *pos, double *normals, double *s, int64_t *sweep,
                         int32_t mem_kind)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    if (mem_kind != SRM_MEM_HOST && mem_kind != SRM_MEM_DEVICE)
        return fail(SRM_EINVAL, "bad mem_kind");
    if (normals && !c->plate) return fail(SRM_EINVAL, "no normals in a ball system");
    const size_t n = (size_t)c->n;
    const hipMemcpyKind kind = (mem_kind == SRM_MEM_HOST) ? hipMemcpyDeviceToHost
                                                          : hipMemcpyDeviceToDevice;
    if (pos) {
        const double *xs[3] = {c->P.x[0], c->P.x[1], c->P.x[2]};
        HIP_TRY(to_id_order(xs, c->dim, c->P.id, c->n, c->dtmp, c->stream));
        HIP_TRY(hipMemcpyAsync(pos, c->dtmp, (size_t)c->dim * n * sizeof(double), kind,
                               c->stream));
    }
    if (normals) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        const double *ns[3] = {c->P.nrm[0], c->P.nrm[1], c->P.nrm[2]};
        HIP_TRY(to_id_order(ns, 3, c->P.id, c->n, c->dtmp, c->stream));
        HIP_TRY(hipMemcpyAsync(normals, c->dtmp, 3 * n * sizeof(double), kind, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (s) *s = c->s;
    if (sweep) *sweep = c->t;
    return SRM_OK;
}

srm_status srm_set_state(srm_ctx *c, const double *pos, const double *normals,
                         int32_t mem_kind)
{
    if (!c || !pos) return fail(SRM_EINVAL, "NULL argument");
    if (mem_kind != SRM_MEM_HOST && mem_kind != SRM_MEM_DEVICE)
        return fail(SRM_EINVAL, "bad mem_kind");
    if (c->plate != (normals != nullptr)) return fail(SRM_EINVAL, "normals iff platelets");
    const size_t n = (size_t)c->n;
    const hipMemcpyKind kind = (mem_kind == SRM_MEM_HOST) ? hipMemcpyHostToDevice
                                                          : hipMemcpyDeviceToDevice;
    // T <- input in id order (rho copied from P in id order first)
    if (c->poly) {
        const double *r[1] = {c->P.rho};
        HIP_TRY(to_id_order(r, 1, c->P.id, c->n, c->dtmp, c->stream));
        HIP_TRY(hipMemcpyAsync(c->T.rho, c->dtmp, n * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    }
    for (int a = 0; a < c->dim; ++a)
        HIP_TRY(hipMemcpyAsync(c->T.x[a], pos + a * n, n * sizeof(double), kind, c->stream));
    if (normals)
        for (int a = 0; a < 3; ++a)
            HIP_TRY(hipMemcpyAsync(c->T.nrm[a], normals + a * n, n * sizeof(double), kind,
                                   c->stream));
    HIP_TRY(launch_iota(c->T.id, c->n, c->stream));
    const Grid g = make_grid(c, c->s * c->rho_max);
    HIP_TRY(launch_zero_counters(c->dcnt, c->stream));
    srm_status st = bin(c, c->T, c->Q, g);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->hcnt->bad) return fail(SRM_EINVAL, "a coordinate is outside [0, L) or NaN");
    std::swap(c->P, c->Q);
    c->acc_valid = false;
    return SRM_OK;
}

srm_status srm_grid(srm_ctx *c, double s, int32_t na[3])
{
    if (!c || !na) return fail(SRM_EINVAL, "NULL argument");
    const Grid g = make_grid(c, s * c->rho_max);
    for (int a = 0; a < 3; ++a) na[a] = g.na[a];
    return SRM_OK;
}

srm_status srm_cells(srm_ctx *c, double grid_s, int32_t *cell_by_id)
{
    if (!c || !cell_by_id) return fail(SRM_EINVAL, "NULL argument");
    const Grid g = make_grid(c, grid_s * c->rho_max);
    HIP_TRY(cells_by_id(c->dim, c->P, c->n, g, c->itmp, c->stream));
    HIP_TRY(hipMemcpyAsync(cell_by_id, c->itmp, (size_t)c->n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SRM_OK;
}

srm_status srm_pass(srm_ctx *c, double grid_s, double radius_s, int32_t kind, int32_t k,
                    uint8_t *acc_by_id, int32_t *overlap)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    if (kind != SRM_PASS_MAIN && kind != SRM_PASS_SHAKE) return fail(SRM_EINVAL, "bad kind");
    if (k < 0 || k > 32767) return fail(SRM_EINVAL, "k out of range");
    const Grid g = make_grid(c, grid_s * c->rho_max);
    srm_status st;
    if ((st = bin(c, c->P, c->T, g))) return st;
    std::swap(c->P, c->T);
    int32_t ov = 0;
    if ((st = run_pass(c, c->P, g, radius_s, kind, k, true, &ov, nullptr))) return st;
    if (overlap) *overlap = ov;
    if (acc_by_id) return srm_last_acc(c, acc_by_id);
    return SRM_OK;
}

srm_status srm_last_acc(srm_ctx *c, uint8_t *acc_by_id)
{
    if (!c || !acc_by_id) return fail(SRM_EINVAL, "NULL argument");
    if (!c->acc_valid) return fail(SRM_EINVAL, "no pass has run");
    uint8_t *tmp = (uint8_t *)c->itmp;
    HIP_TRY(u8_to_id_order(c->acc, c->acc_buf.id, c->n, tmp, c->stream));
    HIP_TRY(hipMemcpyAsync(acc_by_id, tmp, (size_t)c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SRM_OK;
}

namespace {

// Device staging for the diagnostics: copy host inputs in, run, copy out.
struct DevArena {
    void *p[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    ~DevArena()
    {
        for (void *q : p)
            if (q) (void)hipFree(q);
    }
};

}  // namespace

namespace {

// Grid for a static neighbour search with cutoff `reach`: cells at least
// `reach` wide, N_a >= 4 or a single cell per axis, capped like the sweep grid.
Grid cutoff_grid(const srm_ctx *c, double reach)
{
    Grid g{};
    for (int a = 0; a < 3; ++a) {
        g.box[a] = c->p.box[a];
        g.half[a] = 0.5 * c->p.box[a];
        if (a >= c->dim) {
            g.na[a] = 1;
            g.inv_w[a] = 1.0 / c->p.box[a];
            continue;
        }
        int64_t m;
        const double q = (reach > 0.0) ? c->p.box[a] / reach : 0.0;
        if (!(reach > 0.0) || q >= (double)c->ncap) m = c->ncap;
        else m = (int64_t)q;
        g.na[a] = (int32_t)((m >= 4) ? m : 1);
        g.inv_w[a] = (double)g.na[a] / c->p.box[a];
    }
    g.ncell = g.na[0] * g.na[1] * g.na[2];
    return g;
}

// Per-id row counts and offsets for srm_pairs (allocated on first use).
srm_status ensure_rows(srm_ctx *c)
{
    if (c->rowcnt) return SRM_OK;
    hipError_t e;
    if ((e = c->alloc(&c->rowcnt, (size_t)c->n + 2)) || (e = c->alloc(&c->rowoff, (size_t)c->n + 2)) ||
        (e = c->alloc(&c->dsum, 1)))
        return fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    return SRM_OK;
}

// Pairs counted per particle (rowcnt) summed in 64 bits.  The row offsets
// and pair indices downstream are int32, so a total beyond 2^31 - 1 is
// refused here, before any scan or emit kernel runs.
srm_status pair_total(srm_ctx *c, int64_t *total)
{
    HIP_TRY(sum_counts64(c->rowcnt, c->n, c->dsum, c->stream));
    unsigned long long t = 0;
    HIP_TRY(hipMemcpyAsync(&t, c->dsum, sizeof t, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *total = (int64_t)t;
    if (t > (unsigned long long)INT32_MAX)
        return fail(SRM_ECAPACITY, "%llu pairs: more than 2^31 - 1", t);
    return SRM_OK;
}

srm_status check_gap(const srm_ctx *c, double gap)
{
    if (!(gap >= 0.0) || !isfinite(gap)) return fail(SRM_EINVAL, "gap must be finite and >= 0");
    double lmin = c->p.box[0];
    for (int a = 1; a < c->dim; ++a) lmin = c->p.box[a] < lmin ? c->p.box[a] : lmin;
    if (!(2.0 * (c->s * c->rho_max) + gap <= 0.5 * lmin))
        return fail(SRM_EINVAL, "2 R_max + gap must not exceed half the box");
    return SRM_OK;
}

}  // namespace

srm_status srm_pairs(srm_ctx *c, double gap, int64_t cap, int32_t *ij, int64_t *count,
                     int32_t mem_kind)
{
    if (!c || !count) return fail(SRM_EINVAL, "NULL argument");
    srm_status st = check_gap(c, gap);
    if (st) return st;
    if (mem_kind != SRM_MEM_HOST && mem_kind != SRM_MEM_DEVICE)
        return fail(SRM_EINVAL, "bad mem_kind");
    if (cap < 0 || (cap > 0 && !ij)) return fail(SRM_EINVAL, "bad output buffer");
    if ((st = ensure_rows(c))) return st;
    const double reach = 2.0 * (c->s * c->rho_max) + gap;
    const Grid g = cutoff_grid(c, reach);
    if ((st = bin(c, c->P, c->T, g))) return st;
    HIP_TRY(pairs_count(c->dim, c->T, c->sc.start, g, c->n, c->kshape, c->tau, c->s, gap, c->rowcnt,
                        c->stream));
    int64_t total = 0;
    st = pair_total(c, &total);
    *count = total;
    if (st) return st;
    if (total > cap)
        return fail(SRM_ECAPACITY, "%lld pairs exceed capacity %lld", (long long)total,
                    (long long)cap);
    if (total == 0) return SRM_OK;
    HIP_TRY(scan_counts(c->rowcnt, c->rowoff, c->sc.partials, c->n, c->stream));
    DevArena d;
    HIP_TRY(hipMalloc(&d.p[0], (size_t)total * sizeof(int32_t)));
    int32_t *out = ij;
    if (mem_kind == SRM_MEM_HOST) {
        HIP_TRY(hipMalloc(&d.p[1], (size_t)total * 2 * sizeof(int32_t)));
        out = (int32_t *)d.p[1];
    }
    HIP_TRY(pairs_emit(c->dim, c->T, c->sc.start, g, c->n, c->kshape, c->tau, c->s, gap, c->rowoff,
                       (int32_t *)d.p[0], out, c->stream));
    if (mem_kind == SRM_MEM_HOST)
        HIP_TRY(hipMemcpyAsync(ij, out, (size_t)total * 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                               c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SRM_OK;
}

srm_status srm_rdf(srm_ctx *c, int32_t nbins, double r_max, uint64_t *counts, double *g_out)
{
    if (!c || !counts) return fail(SRM_EINVAL, "NULL argument");
    if (nbins < 1 || nbins > 65536) return fail(SRM_EINVAL, "nbins out of range");
    double lmin = c->p.box[0];
    for (int a = 1; a < c->dim; ++a) lmin = c->p.box[a] < lmin ? c->p.box[a] : lmin;
    if (!(r_max > 0.0) || !(r_max <= 0.5 * lmin)) return fail(SRM_EINVAL, "need 0 < r_max <= L/2");
    const Grid g = cutoff_grid(c, r_max);
    srm_status st;
    if ((st = bin(c, c->P, c->T, g))) return st;
    DevArena d;
    HIP_TRY(hipMalloc(&d.p[0], (size_t)nbins * sizeof(uint64_t)));
    HIP_TRY(launch_fill_i32((int32_t *)d.p[0], 2 * (int64_t)nbins, 0, c->stream));
    const double inv = (double)nbins / r_max;
    HIP_TRY(rdf_counts(c->dim, c->T, c->sc.start, g, c->n, nbins, inv,
                       (unsigned long long *)d.p[0], c->stream));
    HIP_TRY(hipMemcpyAsync(counts, d.p[0], (size_t)nbins * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (g_out) {
        double vbox = 1.0;
        for (int a = 0; a < c->dim; ++a) vbox *= c->p.box[a];
        const double coeff = (c->dim == 2) ? M_PI : 4.0 * M_PI / 3.0;
        const double npairs = 0.5 * (double)c->n * (double)(c->n - 1);
        const double dr = r_max / nbins;
        for (int32_t b = 0; b < nbins; ++b) {
            const double r0 = b * dr, r1 = (b + 1) * dr;
            const double shell = (c->dim == 2) ? coeff * (r1 * r1 - r0 * r0)
                                               : coeff * (r1 * r1 * r1 - r0 * r0 * r0);
            const double ideal = npairs * shell / vbox;
            g_out[b] = ideal > 0.0 ? (double)counts[b] / ideal : 0.0;
        }
    }
    return SRM_OK;
}

namespace {

// Wrapping axes (bit a) of the clusters of particles that overlap after
// growing by `gap`.
srm_status percolation_mask(srm_ctx *c, double gap, int32_t *mask)
{
    srm_status st = ensure_rows(c);
    if (st) return st;
    const double reach = 2.0 * (c->s * c->rho_max) + gap;
    const Grid g = cutoff_grid(c, reach);
    if ((st = bin(c, c->P, c->T, g))) return st;
    HIP_TRY(pairs_count(c->dim, c->T, c->sc.start, g, c->n, c->kshape, c->tau, c->s, gap, c->rowcnt,
                        c->stream));
    int64_t total = 0;
    if ((st = pair_total(c, &total))) return st;
    *mask = 0;
    if (total == 0) return SRM_OK;
    HIP_TRY(scan_counts(c->rowcnt, c->rowoff, c->sc.partials, c->n, c->stream));
    DevArena d;
    HIP_TRY(hipMalloc(&d.p[0], (size_t)total * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&d.p[1], (size_t)total * 2 * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&d.p[2], (size_t)total * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&d.p[3], (size_t)c->n * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&d.p[4], 4 * sizeof(int32_t)));
    int32_t *ij = (int32_t *)d.p[1], *shift = (int32_t *)d.p[2], *flags = (int32_t *)d.p[4];
    auto *state = (unsigned long long *)d.p[3];
    HIP_TRY(pairs_emit(c->dim, c->T, c->sc.start, g, c->n, c->kshape, c->tau, c->s, gap, c->rowoff,
                       (int32_t *)d.p[0], ij, c->stream));
    const double *xs[3] = {c->P.x[0], c->P.x[1], c->P.x[2]};
    HIP_TRY(to_id_order(xs, c->dim, c->P.id, c->n, c->dtmp, c->stream));
    HIP_TRY(bond_shifts(ij, total, c->dtmp, c->n, c->dim, g, shift, c->stream));
    HIP_TRY(perc_init(state, c->n, c->stream));
    HIP_TRY(launch_fill_i32(flags, 4, 0, c->stream));
    int32_t host[4] = {0, 0, 0, 0};
    // each round moves every cluster's smallest label at least one bond further
    for (int64_t round = 0;; ++round) {
        if (round > (int64_t)c->n + 1) return fail(SRM_EDEVICE, "percolation labels did not settle");
        HIP_TRY(launch_fill_i32(flags, 1, 0, c->stream));
        HIP_TRY(perc_relax(ij, shift, total, state, flags, c->stream));
        HIP_TRY(hipMemcpyAsync(host, flags, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (host[1]) return fail(SRM_ECAPACITY, "cluster image offsets exceed the packed range");
        if (!host[0]) break;
    }
    HIP_TRY(perc_check(ij, shift, total, state, flags, c->stream));
    HIP_TRY(hipMemcpyAsync(host, flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *mask = host[2];
    return SRM_OK;
}

}  // namespace

srm_status srm_percolation(srm_ctx *c, double gap, int32_t *wraps)
{
    if (!c || !wraps) return fail(SRM_EINVAL, "NULL argument");
    srm_status st = check_gap(c, gap);
    if (st) return st;
    return percolation_mask(c, gap, wraps);
}

srm_status srm_critical_gap(srm_ctx *c, double lo, double hi, int32_t iters, double *gap_c)
{
    if (!c || !gap_c) return fail(SRM_EINVAL, "NULL argument");
    if (iters < 0 || iters > 200 || !(lo < hi)) return fail(SRM_EINVAL, "need lo < hi, 0 <= iters <= 200");
    srm_status st;
    if ((st = check_gap(c, lo)) || (st = check_gap(c, hi))) return st;
    int32_t m_lo = 0, m_hi = 0;
    if ((st = percolation_mask(c, lo, &m_lo)) || (st = percolation_mask(c, hi, &m_hi))) return st;
    if (m_lo || !m_hi) return fail(SRM_EINVAL, "lo must not percolate and hi must");
    for (int32_t k = 0; k < iters; ++k) {
        const double mid = 0.5 * (lo + hi);
        int32_t m = 0;
        if ((st = percolation_mask(c, mid, &m))) return st;
        if (m) hi = mid;
        else lo = mid;
    }
    *gap_c = hi;
    return SRM_OK;
}

srm_status srm_nearest(srm_ctx *c, double r_max, double *dist_by_id, int32_t nbins,
                       uint64_t *hist)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    if (c->p.shape != SRM_BALL) return fail(SRM_EINVAL, "nearest neighbours are for balls");
    if (hist && (nbins < 1 || nbins > 65536)) return fail(SRM_EINVAL, "nbins out of range");
    double lmin = c->p.box[0];
    for (int a = 1; a < c->dim; ++a) lmin = c->p.box[a] < lmin ? c->p.box[a] : lmin;
    if (!(r_max > 0.0) || !(r_max <= 0.5 * lmin)) return fail(SRM_EINVAL, "need 0 < r_max <= L/2");
    const Grid g = cutoff_grid(c, r_max);
    srm_status st;
    if ((st = bin(c, c->P, c->T, g))) return st;
    DevArena d;
    if (dist_by_id) HIP_TRY(hipMalloc(&d.p[0], (size_t)c->n * sizeof(double)));
    if (hist) {
        HIP_TRY(hipMalloc(&d.p[1], (size_t)nbins * sizeof(uint64_t)));
        HIP_TRY(launch_fill_i32((int32_t *)d.p[1], 2 * (int64_t)nbins, 0, c->stream));
    }
    HIP_TRY(nearest(c->dim, c->T, c->sc.start, g, c->n, r_max, (double *)d.p[0], nbins,
                    (unsigned long long *)d.p[1], c->stream));
    if (dist_by_id)
        HIP_TRY(hipMemcpyAsync(dist_by_id, d.p[0], (size_t)c->n * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
    if (hist)
        HIP_TRY(hipMemcpyAsync(hist, d.p[1], (size_t)nbins * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SRM_OK;
}

srm_status srm_profile_enable(srm_ctx *c, int32_t on)
{
    if (!c) return fail(SRM_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->resolve();
    c->prof = srm_profile{};
    c->prof_on = (on & 1) != 0;
    c->count_trials_on = (on & 2) != 0;
    HIP_TRY(launch_fill_i32((int32_t *)c->dtrials, 2, 0, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SRM_OK;
}

srm_status srm_profile_read(srm_ctx *c, srm_profile *out)
{
    if (!c || !out) return fail(SRM_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->resolve();
    unsigned long long trials = 0;
    HIP_TRY(hipMemcpy(&trials, c->dtrials, sizeof(trials), hipMemcpyDeviceToHost));
    c->prof.trials = (int64_t)trials;
    *out = c->prof;
    return SRM_OK;
}


srm_status srm_debug_fp(const double *a, const double *b, int64_t n, double *sqrt_out,
                        double *div_out)
{
    if (n < 0 || n > 0x7fffffffLL || (n > 0 && (!a || !b || !sqrt_out || !div_out)))
        return fail(SRM_EINVAL, "bad arguments");
    if (n == 0) return SRM_OK;
    DevArena d;
    const size_t bytes = (size_t)n * sizeof(double);
    for (int i = 0; i < 4; ++i) HIP_TRY(hipMalloc(&d.p[i], bytes));
    HIP_TRY(hipMemcpy(d.p[0], a, bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.p[1], b, bytes, hipMemcpyHostToDevice));
    HIP_TRY(diag_fp((double *)d.p[0], (double *)d.p[1], (int32_t)n, (double *)d.p[2],
                    (double *)d.p[3], nullptr));
    HIP_TRY(hipMemcpy(sqrt_out, d.p[2], bytes, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(div_out, d.p[3], bytes, hipMemcpyDeviceToHost));
    return SRM_OK;
}

srm_status srm_debug_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out)
{
    if (n < 0 || n > 0x0fffffffLL || (n > 0 && (!ctr || !key || !out)))
        return fail(SRM_EINVAL, "bad arguments");
    if (n == 0) return SRM_OK;
    DevArena d;
    HIP_TRY(hipMalloc(&d.p[0], (size_t)n * 16));
    HIP_TRY(hipMalloc(&d.p[1], (size_t)n * 8));
    HIP_TRY(hipMalloc(&d.p[2], (size_t)n * 16));
    HIP_TRY(hipMemcpy(d.p[0], ctr, (size_t)n * 16, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.p[1], key, (size_t)n * 8, hipMemcpyHostToDevice));
    HIP_TRY(diag_philox((const uint32_t *)d.p[0], (const uint32_t *)d.p[1], (int32_t)n,
                        (uint32_t *)d.p[2], nullptr));
    HIP_TRY(hipMemcpy(out, d.p[2], (size_t)n * 16, hipMemcpyDeviceToHost));
    return SRM_OK;
}

srm_status srm_debug_unitvec(int32_t dim, uint64_t seed, uint32_t t, uint32_t word,
                             uint32_t stream, double len, int64_t n, double *out)
{
    if ((dim != 2 && dim != 3) || n < 0 || n > 0x0fffffffLL || (n > 0 && !out))
        return fail(SRM_EINVAL, "bad arguments");
    if (n == 0) return SRM_OK;
    DevArena d;
    HIP_TRY(hipMalloc(&d.p[0], (size_t)n * 24));
    HIP_TRY(diag_unitvec(dim, seed, t, word, stream, len, (int32_t)n, (double *)d.p[0], nullptr));
    HIP_TRY(hipMemcpy(out, d.p[0], (size_t)n * 24, hipMemcpyDeviceToHost));
    return SRM_OK;
}

// ---------------------------------------------------------------- soft g(r)

}  // extern "C"

struct srm_soft {
    srm_softrdf_params p{};
    int32_t n = 0;
    hipStream_t stream = nullptr;
    int64_t ncap = 0;
    PBuf in{}, sorted{};
    Scratch sc{};
    Counters *dcnt = nullptr;
    double *partial = nullptr;
    Grid g{};
    std::vector<void *> allocs;
    template <class T_>
    hipError_t alloc(T_ **ptr, size_t count)
    {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, (count > 0 ? count : 1) * sizeof(T_));
        if (e == hipSuccess) {
            allocs.push_back(v);
            *ptr = (T_ *)v;
        }
        return e;
    }
    ~srm_soft()
    {
        for (void *v : allocs) (void)hipFree(v);
    }
};

namespace {

// Validates the descriptor's parameters (dim, bins, cutoff, box) for n
// particles and builds its neighbour grid: cells at least r_c + 4h wide,
// capped like the SRM grid.  pp is *p with box[2] = 1 in 2D.
srm_status soft_setup(const srm_softrdf_params *p, int64_t n, srm_softrdf_params &pp, Grid &g)
{
    if (!p) return fail(SRM_EINVAL, "NULL argument");
    if (p->dim != 2 && p->dim != 3) return fail(SRM_EINVAL, "dim must be 2 or 3");
    if (p->nbins < 1 || p->nbins > 64) return fail(SRM_EINVAL, "nbins must be 1..64");
    if (n < 2 || n > 0x7fffffffLL) return fail(SRM_EINVAL, "n out of range");
    if (!(p->r_c > 0.0) || !isfinite(p->r_c) || !(p->kappa >= 0.0))
        return fail(SRM_EINVAL, "bad r_c or kappa");
    for (int a = 0; a < p->dim; ++a)
        if (!(p->box[a] > 0.0)) return fail(SRM_EINVAL, "box edge <= 0");
    pp = *p;
    if (pp.dim == 2) pp.box[2] = 1.0;
    const int64_t ncap = cell_cap(pp.dim, n);
    const double cut = pp.r_c + 4.0 * (pp.r_c / pp.nbins);
    for (int a = 0; a < 3; ++a) {
        g.box[a] = pp.box[a];
        g.half[a] = 0.5 * pp.box[a];
        if (a >= pp.dim) {
            g.na[a] = 1;
            g.inv_w[a] = 1.0 / pp.box[a];
            continue;
        }
        const double q = pp.box[a] / cut;
        const int64_t m = (q >= (double)ncap) ? ncap : (int64_t)q;
        g.na[a] = (int32_t)(m >= 4 ? m : 1);
        g.inv_w[a] = (double)g.na[a] / pp.box[a];
    }
    g.ncell = g.na[0] * g.na[1] * g.na[2];
    return SRM_OK;
}

srm_status soft_bin(srm_soft *c, const double *pos, const double *radii)
{
    const size_t n = (size_t)c->n;
    for (int a = 0; a < c->p.dim; ++a)
        HIP_TRY(hipMemcpyAsync(c->in.x[a], pos + a * n, n * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->in.rho, radii, n * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    HIP_TRY(launch_iota(c->in.id, c->n, c->stream));
    HIP_TRY(bin_particles(c->p.dim, c->in, c->sorted, c->n, c->g, c->sc, c->dcnt, c->stream));
    return SRM_OK;
}

}  // namespace

extern "C" {

srm_status srm_softrdf_create(const srm_softrdf_params *p, int64_t n, void *stream,
                              srm_soft **out)
{
    if (!out) return fail(SRM_EINVAL, "NULL argument");
    srm_softrdf_params pp{};
    Grid g{};
    const srm_status st = soft_setup(p, n, pp, g);
    if (st) return st;
    srm_soft *c = new (std::nothrow) srm_soft();
    if (!c) return fail(SRM_ENOMEM, "host allocation failed");
    c->p = pp;
    c->n = (int32_t)n;
    c->stream = (hipStream_t)stream;
    c->ncap = cell_cap(c->p.dim, n);
    c->g = g;
    hipError_t e = hipSuccess;
    for (int a = 0; a < c->p.dim && !e; ++a)
        if ((e = c->alloc(&c->in.x[a], n)) == hipSuccess) e = c->alloc(&c->sorted.x[a], n);
    if (!e) e = c->alloc(&c->in.id, n);
    if (!e) e = c->alloc(&c->sorted.id, n);
    if (!e) e = c->alloc(&c->in.rho, n);
    if (!e) e = c->alloc(&c->sorted.rho, n);
    c->sc.cap = n + 2;
    if (!e) e = c->alloc(&c->sc.cell, n);
    if (!e) e = c->alloc(&c->sc.slot, n);
    if (!e) e = c->alloc(&c->sc.tmpid, n);
    if (!e) e = c->alloc(&c->sc.counts, (size_t)c->sc.cap);
    if (!e) e = c->alloc(&c->sc.start, (size_t)c->sc.cap + 1);
    if (!e) e = c->alloc(&c->sc.partials, (size_t)(c->sc.cap / 2048 + 2));
    if (!e) e = c->alloc(&c->dcnt, 1);
    if (!e) e = c->alloc(&c->partial, (size_t)soft_blocks(c->n) * soft_partial_stride());
    if (e) {
        delete c;
        return fail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return SRM_OK;
}

srm_status srm_softrdf_forward(srm_soft *c, const double *pos, const double *radii,
                               double *g_out, double *energy)
{
    if (!c || !pos || !radii || !g_out || !energy) return fail(SRM_EINVAL, "NULL argument");
    srm_status st = soft_bin(c, pos, radii);
    if (st) return st;
    HIP_TRY(soft_forward(c->p.dim, c->sorted, c->sc.start, c->g, c->n, c->p.nbins, c->p.r_c,
                         c->p.kappa, c->partial, g_out, energy, c->stream));
    return SRM_OK;
}

srm_status srm_softrdf_backward(srm_soft *c, const double *pos, const double *radii,
                                const double *dg, const double *dE, double *grad_pos,
                                double *grad_radii)
{
    if (!c || !pos || !radii || !dg || !dE || !grad_pos || !grad_radii)
        return fail(SRM_EINVAL, "NULL argument");
    srm_status st = soft_bin(c, pos, radii);
    if (st) return st;
    HIP_TRY(soft_backward(c->p.dim, c->sorted, c->sc.start, c->g, c->n, c->p.nbins, c->p.r_c,
                          c->p.kappa, dg, dE, grad_pos, grad_radii, c->stream));
    return SRM_OK;
}

srm_status srm_softrdf_free(srm_soft *c)
{
    if (!c) return SRM_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete c;
    return SRM_OK;
}

}  // extern "C"

// ------------------------------------------- soft g(r) without allocation
//
// srm_softrdf_forward_static runs the forward above on a file-scope device
// array instead of a workspace: cell-sorted copies of positions, radii and
// ids, the id sequence, the binning scratch, the scan partials, the
// counters and the block partials, for at most kStaticSoftN particles.
// Each device holds its own copy of the array; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.

namespace {

constexpr int64_t kStaticSoftN = SRM_SOFTRDF_STATIC_MAX_N;

constexpr size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

struct StaticSoftLayout {
    size_t x[3], rho, id, inid, cell, slot, tmpid, counts, start, partials, cnt, partial, total;
};

constexpr StaticSoftLayout static_soft_layout(int64_t n)
{
    StaticSoftLayout L{};
    const size_t un = (size_t)n, cap = un + 2;
    size_t o = 0;
    for (int a = 0; a < 3; ++a) {
        L.x[a] = o;
        o += up256(un * sizeof(double));
    }
    L.rho = o;
    o += up256(un * sizeof(double));
    L.id = o;
    o += up256(un * sizeof(int32_t));
    L.inid = o;
    o += up256(un * sizeof(int32_t));
    L.cell = o;
    o += up256(un * sizeof(int32_t));
    L.slot = o;
    o += up256(un * sizeof(int32_t));
    L.tmpid = o;
    o += up256(un * sizeof(int32_t));
    L.counts = o;
    o += up256(cap * sizeof(int32_t));
    L.start = o;
    o += up256((cap + 1) * sizeof(int32_t));
    L.partials = o;
    o += up256((cap / 2048 + 2) * sizeof(int32_t));
    L.cnt = o;
    o += up256(sizeof(Counters));
    L.partial = o;
    o += up256((un + kSoftBlock - 1) / kSoftBlock * kSoftPartialStride * sizeof(double));
    L.total = o;
    return L;
}

constexpr size_t kStaticSoftBytes = static_soft_layout(kStaticSoftN).total;

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
unsigned char *g_static_base[kMaxDevices];  // device address of `scratch`, per device

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticSoftBytes];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (the array's name is not a device address in host code).
srm_status static_scratch(unsigned char **base)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SRM_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SRM_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_base[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SRM_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_static_base[dev] = (unsigned char *)ptr;
    }
    *base = g_static_base[dev];
    return SRM_OK;
}

}  // namespace

extern "C" {

srm_status srm_softrdf_forward_static(const srm_softrdf_params *p, int64_t n, const double *pos,
                                      const double *radii, double *g_out, double *energy,
                                      void *stream)
{
    if (!pos || !radii || !g_out || !energy) return fail(SRM_EINVAL, "NULL argument");
    srm_softrdf_params pp{};
    Grid g{};
    srm_status st = soft_setup(p, n, pp, g);
    if (st) return st;
    if (n > kStaticSoftN)
        return fail(SRM_ECAPACITY, "n = %lld exceeds the static workspace of %lld particles",
                    (long long)n, (long long)kStaticSoftN);
    unsigned char *base = nullptr;
    if ((st = static_scratch(&base))) return st;
    constexpr StaticSoftLayout L = static_soft_layout(kStaticSoftN);
    const hipStream_t s = (hipStream_t)stream;
    const int32_t nn = (int32_t)n;
    PBuf in{}, sorted{};
    for (int a = 0; a < pp.dim; ++a) {
        in.x[a] = const_cast<double *>(pos + (size_t)a * (size_t)n);
        sorted.x[a] = (double *)(base + L.x[a]);
    }
    in.rho = const_cast<double *>(radii);
    in.id = (int32_t *)(base + L.inid);
    sorted.rho = (double *)(base + L.rho);
    sorted.id = (int32_t *)(base + L.id);
    Scratch sc{};
    sc.cell = (int32_t *)(base + L.cell);
    sc.slot = (int32_t *)(base + L.slot);
    sc.tmpid = (int32_t *)(base + L.tmpid);
    sc.counts = (int32_t *)(base + L.counts);
    sc.start = (int32_t *)(base + L.start);
    sc.partials = (int32_t *)(base + L.partials);
    sc.cap = n + 2;
    Counters *cnt = (Counters *)(base + L.cnt);
    double *partial = (double *)(base + L.partial);
    HIP_TRY(launch_iota(in.id, nn, s));
    HIP_TRY(launch_zero_counters(cnt, s));
    HIP_TRY(bin_particles(pp.dim, in, sorted, nn, g, sc, cnt, s));
    HIP_TRY(soft_forward(pp.dim, sorted, sc.start, g, nn, pp.nbins, pp.r_c, pp.kappa, partial,
                         g_out, energy, s));
    return SRM_OK;
}

}  // extern "C"
