// zda_runtime.hip -- host runtime of the ZDA zone library: the C ABI of
// include/zda.h.  Zone setup (FP64 precompute of the per-row metric and PML
// constants, device allocation), the time loop, the broadband adjoint source
// and the gradient overlap (arXiv 2501.07979, section on the cylindrical
// solver and eq. 6).  All per-cell work runs in zda_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <array>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "zda_internal.h"

using cd = std::complex<double>;
using namespace zda;

namespace {

thread_local std::string g_last_error;

zda_status fail(zda_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(ZDA_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// graded conductivity at coordinate p (cell units) on an axis of n cells
double grade(double p, int n, int d0, int d1, double order, double smax)
{
    double rho = 0.0;
    if (d0 > 0 && p < d0) rho = (d0 - p) / d0;
    else if (d1 > 0 && p > n - d1) rho = (p - (n - d1)) / d1;
    return rho > 0.0 ? smax * std::pow(rho, order) : 0.0;
}

// The device allocator registered with zda_set_allocator (NULL functions:
// hipMalloc / hipFree).  Zones and batches copy it when they are created.
struct Allocator {
    zda_alloc_fn alloc = nullptr;
    zda_free_fn free = nullptr;
    void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator()
{
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    return g_alloc;
}

// Device memory owned by one zone or batch: every buffer with its size,
// returned through the allocator that made it.
struct DevMem {
    Allocator al;
    int device = 0;
    std::vector<std::pair<void *, size_t>> live;
    size_t bytes = 0;

    void *get(size_t n)
    {
        void *p = nullptr;
        if (al.alloc) {
            p = al.alloc(n, device, al.ctx);
        } else if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p) {
            live.push_back({p, n});
            bytes += n;
        }
        return p;
    }
    void release(void *p, size_t n)
    {
        if (al.free) al.free(p, n, device, al.ctx);
        else (void)hipFree(p);
    }
    void put(void *p)
    {
        if (!p) return;
        for (size_t q = 0; q < live.size(); ++q)
            if (live[q].first == p) {
                release(p, live[q].second);
                bytes -= live[q].second;
                live[q] = live.back();
                live.pop_back();
                return;
            }
    }
    void put_all()
    {
        for (auto &e : live) release(e.first, e.second);
        live.clear();
        bytes = 0;
    }
};

// Pinned host staging of one zone's (or batch's) uploads: a ring of slots,
// each rewritten only after the copies that read it last (marked by its
// event) have run, so a call never waits for the work of the call before.
struct Stage {
    static constexpr int N = 6;
    void *buf[N] = {};
    size_t cap[N] = {};
    hipEvent_t ev[N] = {};
    bool pending[N] = {};
    int next = 0, cur = -1;

    // a slot of at least n bytes that is free for writing
    void *take(size_t n)
    {
        const int q = next;
        next = (next + 1) % N;
        if (pending[q]) {
            if (hipEventSynchronize(ev[q]) != hipSuccess) return nullptr;
            pending[q] = false;
        }
        if (!ev[q] && hipEventCreateWithFlags(&ev[q], hipEventDisableTiming) != hipSuccess) return nullptr;
        if (cap[q] < n) {
            if (buf[q]) (void)hipHostFree(buf[q]);
            buf[q] = nullptr;
            cap[q] = 0;
            const size_t want = std::max(n, (size_t)1 << 16);
            if (hipHostMalloc(&buf[q], want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                buf[q] = nullptr;
                return nullptr;
            }
            cap[q] = want;
        }
        cur = q;
        return buf[q];
    }
    // the copies just enqueued on s read the slot taken last
    hipError_t issued(hipStream_t s)
    {
        if (cur < 0) return hipSuccess;
        hipError_t e = hipEventRecord(ev[cur], s);
        pending[cur] = e == hipSuccess;
        cur = -1;
        return e;
    }
    void destroy()
    {
        for (int q = 0; q < N; ++q) {
            if (pending[q]) (void)hipEventSynchronize(ev[q]);
            if (buf[q]) (void)hipHostFree(buf[q]);
            if (ev[q]) (void)hipEventDestroy(ev[q]);
            buf[q] = nullptr;
            ev[q] = nullptr;
            cap[q] = 0;
            pending[q] = false;
        }
    }
};

// Tile counts of a two-step tile list (interior tiles first, then the layer
// tiles by instantiation) and the cells the interior tiles own.
struct TileCounts {
    unsigned n_lay[N_LAY] = {};
    size_t cells = 0, mon = 0, src = 0;
};

// Device buffers one run stages its inputs in: the zone's own (grown on
// demand), or slices of the library's static scratch array for the entry
// point that allocates nothing.
struct RunBufs {
    bool noalloc = false;
    float2 *pattern = nullptr, *profile = nullptr, *twiddle = nullptr;
    uint4 *tiles = nullptr;
    size_t cap_pattern = 0, cap_profile = 0, cap_twiddle = 0, cap_tiles = 0;   // noalloc: slice sizes
};

// watchdog bound on |F|^2 (|F| = 1e18; FP32 squares overflow near 1.8e19)
constexpr float WATCH_BOUND2 = 1e36f;

}  // namespace

struct zda_zone {
    zda_zone_desc d;
    int device = 0;
    double dt = 0, dphi = 0, tau = 0, cfl = 0;
    size_t ncell = 0, plane = 0;
    int dR = 0, dZ = 0, nd = 0, kchunk = 1, tile_rows = 7;
    // FP64 layer constants: [0] integer points, [1] half points
    std::vector<double> sig_r[2], Sig_r[2], sgt_r[2], sig_z[2];
    // FP64 per-row and per-plane coefficients (the FP32 ones are these rounded)
    std::vector<RowCoefT<double>> rows64;
    std::vector<ZCoefT<double>> zrows64;
    // device state of the FP64 verification runs (allocated by the first one)
    struct F64 {
        double2 *F[6] = {};
        double *ceps = nullptr;
        double2 *auxR = nullptr, *auxZ = nullptr;
        RowCoefT<double> *rows = nullptr;
        ZCoefT<double> *zrows = nullptr;
        double2 *pattern = nullptr, *dft = nullptr, *prof = nullptr, *tw = nullptr;
        size_t cap_steps = 0;
        bool ready = false;
    } f64;
    double cr = 1, cz = 1;
    DevMem mem;
    Stage stage;
    // the stream the zone's work is ordered on: the stream of its last run,
    // or the one given to zda_zone_set_stream
    hipStream_t stream = nullptr;
    // device memory
    // two buffer sets of the six fields and the PML auxiliaries: the split
    // kernels update set `cur` in place, the fused kernel steps cur -> cur^1
    float2 *F[2][6] = {{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},
                       {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}};
    float *ceps = nullptr;
    float2 *auxR[2] = {nullptr, nullptr}, *auxZ[2] = {nullptr, nullptr};
    int cur = 0;
    bool fused = true;
    bool two = false;              // two leap-frog steps per launch (tile_rows 5, 13 or 34)
    int xcd_remap = 0, nt_stores = 1, layer_stream = 0;
    int tile_patch = 0;            // (bands << 8) | columns of an XCD's patch of two-step tiles, 0 = off
    int layer_kchunk = -1;         // planes per chunk of the r-layer band tiles (-1: automatic)
    int layer_carry = 1;           // 1: layer tiles keep step one's auxiliaries in registers
    int watch_every = 1000;        // steps between in-loop divergence checks (0: off)
    int tiles_lkc = -2, tiles_carry = -1;
    // second stream and join events for the concurrent layer-tile launch
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // two-step launches: auxiliaries at the intermediate time level, and the
    // tile lists (interior tiles without layer cells first, then layer tiles)
    float2 *mauxR = nullptr, *mauxZ = nullptr;
    // three-step launches (tile_rows THREE_STEP_ROWS): the second
    // intermediate time level, allocated when the zone first selects them
    float2 *m2auxR = nullptr, *m2auxZ = nullptr;
    bool has_m2 = false, three = false;
    uint4 *tiles2 = nullptr;
    size_t cap_tiles2 = 0;
    bool has_m = false;
    // the time-stepping memory (field sets, auxiliaries, intermediate sets)
    // is given back by zda_zone_release_fields until zda_zone_acquire_fields;
    // has_second: the zone holds a second buffer set whenever it holds any;
    // fields_external: that memory is carved from a caller's buffer
    bool released = false, has_second = false, fields_external = false;
    TileCounts tc;
    int tiles_tr = 0, tiles_kc = 0, tiles_src = -1, k_src_last = -1, tiles_xcd = -1;
    RowCoef *rows = nullptr;
    ZCoef *zrows = nullptr;
    float2 *dft_plane = nullptr, *dft_vol = nullptr, *dft_vol_adj = nullptr;
    float2 *pattern = nullptr, *profile = nullptr, *twiddle = nullptr, *scratch = nullptr;
    size_t cap_pattern = 0, cap_profile = 0, cap_twiddle = 0, cap_scratch = 0;
    int pattern_key = 0;           // preset pattern held in `pattern` (0: none)
    int *flag = nullptr;           // sticky divergence flag (device)
    int *flag_host = nullptr;      // pinned mirror, refreshed by the copies enqueued after runs and reads
    // host staging of the entry point that allocates nothing (pageable)
    std::vector<float2> st_pat, st_prof, st_tw;
    std::vector<uint4> st_tiles;
    // state of the last forward run
    int n_done = 0;
    int last_K = 0;
    double last_omega[ZDA_MAX_FREQ] = {0};
    int last_T = 0;
    double last_width = 0;
    int last_n0 = -1;
    bool have_plane = false, have_vol = false, have_vol_adj = false;
    // per-launch timing events of the last timed run
    std::vector<hipEvent_t> ev;
    int timed_steps = 0;
    bool timed_fused = false;
    bool timed_two = false;
    int timed_depth = 2;
    TileCounts timed_tc;
};

namespace {

template <typename T>
zda_status dev_alloc(zda_zone *z, T **p, size_t count)
{
    if (count == 0) { *p = nullptr; return ZDA_OK; }
    void *q = z->mem.get(count * sizeof(T));
    if (!q) return fail(ZDA_ERR_OOM, "device allocation of %zu bytes failed", count * sizeof(T));
    *p = (T *)q;
    return ZDA_OK;
}

template <typename T>
void dev_free(zda_zone *z, T *&p)
{
    z->mem.put((void *)p);
    p = nullptr;
}

// the second intermediate set of the three-step kernel's layer auxiliaries
zda_status alloc_m2(zda_zone *z)
{
    zda_status st = dev_alloc(z, &z->m2auxR, (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi);
    if (st == ZDA_OK) st = dev_alloc(z, &z->m2auxZ, (size_t)N_AUX_Z * z->dZ * z->plane);
    if (st != ZDA_OK) {
        dev_free(z, z->m2auxR);
        dev_free(z, z->m2auxZ);
    }
    return st;
}

// the time-stepping buffers of a zone: both field sets, the PML
// auxiliaries and the intermediate sets, with their element counts
template <class F>
void for_each_stepping(zda_zone *z, F f)
{
    const size_t nR = (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi, nZ = (size_t)N_AUX_Z * z->dZ * z->plane;
    for (int b = 0; b < (z->has_second ? 2 : 1); ++b) {
        for (auto &p : z->F[b]) f(p, z->ncell);
        f(z->auxR[b], nR);
        f(z->auxZ[b], nZ);
    }
    if (z->has_m) {
        f(z->mauxR, nR);
        f(z->mauxZ, nZ);
    }
    if (z->three) {
        f(z->m2auxR, nR);
        f(z->m2auxZ, nZ);
    }
}

// bytes of a stepping buffer carved from a caller's memory (256 B aligned)
size_t carved_bytes(size_t n) { return (n * sizeof(float2) + 255) / 256 * 256; }

// free the time-stepping memory (or drop the pointers into a caller's buffer)
void free_stepping(zda_zone *z)
{
    if (z->fields_external) {
        for (auto &set : z->F)
            for (auto &f : set) f = nullptr;
        z->auxR[0] = z->auxR[1] = z->auxZ[0] = z->auxZ[1] = nullptr;
        z->mauxR = z->mauxZ = z->m2auxR = z->m2auxZ = nullptr;
        z->fields_external = false;
        return;
    }
    for (auto &set : z->F)
        for (auto &f : set) dev_free(z, f);
    for (int b = 0; b < 2; ++b) {
        dev_free(z, z->auxR[b]);
        dev_free(z, z->auxZ[b]);
    }
    dev_free(z, z->mauxR);
    dev_free(z, z->mauxZ);
    dev_free(z, z->m2auxR);
    dev_free(z, z->m2auxZ);
}

zda_status released_error()
{
    return fail(ZDA_ERR_STATE, "the zone's fields are released (zda_zone_acquire_fields first)");
}

// wait for everything the zone has enqueued (its stream and the layer stream)
hipError_t zone_wait(zda_zone *z)
{
    hipError_t e = hipStreamSynchronize(z->stream);
    if (e == hipSuccess && z->s2) e = hipStreamSynchronize(z->s2);
    return e;
}

template <typename T>
zda_status ensure(zda_zone *z, T **p, size_t *cap, size_t count)
{
    if (count <= *cap) return ZDA_OK;
    if (*p) {
        // work already enqueued may still read the old buffer
        HIP_TRY(zone_wait(z));
        dev_free(z, *p);
        *cap = 0;
    }
    zda_status st = dev_alloc(z, p, count);
    if (st == ZDA_OK) *cap = count;
    return st;
}

void free_all(zda_zone *z)
{
    for (auto e : z->ev) (void)hipEventDestroy(e);
    z->ev.clear();
    if (z->ev_fork) (void)hipEventDestroy(z->ev_fork);
    if (z->ev_join) (void)hipEventDestroy(z->ev_join);
    if (z->s2) (void)hipStreamDestroy(z->s2);
    z->stage.destroy();
    if (z->flag_host) (void)hipHostFree(z->flag_host);
    z->flag_host = nullptr;
    z->mem.put_all();
}

// refresh the pinned mirror of the divergence flag behind the work on s
hipError_t post_flag(zda_zone *z, hipStream_t s)
{
    return hipMemcpyAsync(z->flag_host, z->flag, sizeof(int), hipMemcpyDeviceToHost, s);
}

// s(w) = 1 + sigma F(w), F = dt / (1 - c e^{i w dt})
cd stretch(double sigma, double c, double w, double dt)
{
    cd F = dt / (1.0 - c * std::exp(cd(0.0, w * dt)));
    return 1.0 + sigma * F;
}

// Layer constants and per-row coefficients (the PML contract of the design
// notes): radial lengths dr (1 + sigma F), radii R = r + Sigma F with Sigma
// accumulated outwards in the outer layer and (regularised, |Sigma|) inwards
// in the inner layer, axial lengths dz (1 + sigma_z F).
void setup_layers(zda_zone *z, std::vector<RowCoef> &rows, std::vector<ZCoef> &zr)
{
    const zda_zone_desc &d = z->d;
    const int nr = d.nr, nz = d.nz, d0 = d.pml_r_in, d1 = d.pml_r_out;
    const double smr = d.pml_sigma_max_r > 0 ? d.pml_sigma_max_r : 0.8 * (d.pml_order + 1.0) / d.dr;
    const double smz = d.pml_sigma_max_z > 0 ? d.pml_sigma_max_z : 0.8 * (d.pml_order + 1.0) / d.dz;
    for (int h = 0; h < 2; ++h) {
        z->sig_r[h].assign(nr + 1, 0.0);
        z->Sig_r[h].assign(nr + 1, 0.0);
        z->sgt_r[h].assign(nr + 1, 0.0);
        z->sig_z[h].assign(nz + 1, 0.0);
        for (int i = 0; i <= nr; ++i) z->sig_r[h][i] = grade(i + 0.5 * h, nr, d0, d1, d.pml_order, smr);
        for (int k = 0; k <= nz; ++k)
            z->sig_z[h][k] = grade(k + 0.5 * h, nz, d.pml_z_lo, d.pml_z_hi, d.pml_order, smz);
    }
    // Sigma on the lattice of integer and half points: each step of half a
    // cell adds dr * sigma at the point in between.
    if (d1 > 0) {
        for (int i = nr - d1 + 1; i <= nr; ++i) z->Sig_r[0][i] = z->Sig_r[0][i - 1] + d.dr * z->sig_r[1][i - 1];
        for (int i = nr - d1; i <= nr; ++i)
            z->Sig_r[1][i] = (i > 0 ? z->Sig_r[1][i - 1] : 0.0) + d.dr * z->sig_r[0][i];
    }
    if (d0 > 0) {
        for (int i = d0 - 1; i >= 0; --i) z->Sig_r[0][i] = z->Sig_r[0][i + 1] + d.dr * z->sig_r[1][i];
        for (int i = d0 - 1; i >= 0; --i) z->Sig_r[1][i] = z->Sig_r[1][i + 1] + d.dr * z->sig_r[0][i + 1];
    }
    double worst = 0.0;
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i <= nr; ++i) {
            const double r = d.r_in + (i + 0.5 * h) * d.dr;
            z->sgt_r[h][i] = z->Sig_r[h][i] / r;
            worst = std::max(worst, -z->sgt_r[h][i]);
        }
    const double dt = z->dt;
    z->cr = std::exp(-(d.pml_alpha + 2.0 * worst) * dt);
    z->cz = std::exp(-d.pml_alpha * dt);
    auto g1 = [&](double s) { return 1.0 / (1.0 + s * dt); };
    auto g2 = [&](double s, double c) { return s * c / (1.0 + s * dt); };
    // FP64 rows (kept for the FP64 verification runs), rounded to FP32 for the kernels
    auto &r64 = z->rows64;
    r64.resize(nr);
    for (int i = 0; i < nr; ++i) {
        const double ri = d.r_in + i * d.dr, rh = ri + 0.5 * d.dr;
        RowCoefT<double> &rc = r64[i];
        rc.inv_rdphi_int = 1.0 / (ri * z->dphi);
        rc.inv_rdphi_half = 1.0 / (rh * z->dphi);
        rc.inv_2r_int = 0.5 / ri;
        rc.inv_2r_half = 0.5 / rh;
        rc.g1_s_int = g1(z->sig_r[0][i]);
        rc.g2_s_int = g2(z->sig_r[0][i], z->cr);
        rc.g1_s_half = g1(z->sig_r[1][i]);
        rc.g2_s_half = g2(z->sig_r[1][i], z->cr);
        rc.g1_t_int = g1(z->sgt_r[0][i]);
        rc.g2_t_int = g2(z->sgt_r[0][i], z->cr);
        rc.g1_t_half = g1(z->sgt_r[1][i]);
        rc.g2_t_half = g2(z->sgt_r[1][i], z->cr);
        rc.hz_c1 = (i + 1 < nr ? z->Sig_r[0][i + 1] : 0.0) / (rh * d.dr);
        rc.hz_c0 = z->Sig_r[0][i] / (rh * d.dr);
        rc.ez_c1 = z->Sig_r[1][i] / (ri * d.dr);
        rc.ez_c0 = (i > 0 ? z->Sig_r[1][i - 1] : 0.0) / (ri * d.dr);
    }
    auto &z64 = z->zrows64;
    z64.resize(nz);
    for (int k = 0; k < nz; ++k) {
        z64[k].g1_int = g1(z->sig_z[0][k]);
        z64[k].g2_int = g2(z->sig_z[0][k], z->cz);
        z64[k].g1_half = g1(z->sig_z[1][k]);
        z64[k].g2_half = g2(z->sig_z[1][k], z->cz);
    }
    rows.resize(nr);
    for (int i = 0; i < nr; ++i) {
        const RowCoefT<double> &q = r64[i];
        RowCoef &rc = rows[i];
        rc.inv_rdphi_int = (float)q.inv_rdphi_int;
        rc.inv_rdphi_half = (float)q.inv_rdphi_half;
        rc.inv_2r_int = (float)q.inv_2r_int;
        rc.inv_2r_half = (float)q.inv_2r_half;
        rc.g1_s_int = (float)q.g1_s_int;
        rc.g2_s_int = (float)q.g2_s_int;
        rc.g1_s_half = (float)q.g1_s_half;
        rc.g2_s_half = (float)q.g2_s_half;
        rc.g1_t_int = (float)q.g1_t_int;
        rc.g2_t_int = (float)q.g2_t_int;
        rc.g1_t_half = (float)q.g1_t_half;
        rc.g2_t_half = (float)q.g2_t_half;
        rc.hz_c1 = (float)q.hz_c1;
        rc.hz_c0 = (float)q.hz_c0;
        rc.ez_c1 = (float)q.ez_c1;
        rc.ez_c0 = (float)q.ez_c0;
    }
    zr.resize(nz);
    for (int k = 0; k < nz; ++k) {
        zr[k].g1_int = (float)z64[k].g1_int;
        zr[k].g2_int = (float)z64[k].g2_int;
        zr[k].g1_half = (float)z64[k].g1_half;
        zr[k].g2_half = (float)z64[k].g2_half;
    }
}

StepArgs step_args(zda_zone *z, int m)
{
    StepArgs a{};
    const zda_zone_desc &d = z->d;
    a.nr = d.nr; a.nphi = d.nphi; a.nz = d.nz;
    a.pr0 = d.pml_r_in; a.pr1 = d.pml_r_out; a.pz0 = d.pml_z_lo; a.pz1 = d.pml_z_hi;
    a.dR = z->dR; a.dZ = z->dZ;
    a.dt = (float)z->dt;
    a.inv_dr = (float)(1.0 / d.dr);
    a.inv_dz = (float)(1.0 / d.dz);
    a.cr = (float)z->cr; a.cz = (float)z->cz;
    if (d.n_fold > 0) {
        const double ph = m * z->tau;
        a.seam_p = make_float2((float)std::cos(ph), (float)std::sin(ph));
        a.seam_m = make_float2((float)std::cos(ph), (float)-std::sin(ph));
    } else {   // continuous zone: 1 +- i m (exact i m derivative with dphi = 1)
        a.seam_p = make_float2(1.f, (float)m);
        a.seam_m = make_float2(1.f, (float)-m);
    }
    a.axis = d.axis ? 1 : 0;
    const int s0 = z->cur, s1 = z->cur ^ 1;
    a.Er = z->F[s0][0]; a.Ep = z->F[s0][1]; a.Ez = z->F[s0][2];
    a.Hr = z->F[s0][3]; a.Hp = z->F[s0][4]; a.Hz = z->F[s0][5];
    a.oEr = z->F[s1][0]; a.oEp = z->F[s1][1]; a.oEz = z->F[s1][2];
    a.oHr = z->F[s1][3]; a.oHp = z->F[s1][4]; a.oHz = z->F[s1][5];
    a.ceps = z->ceps;
    a.auxR = z->auxR[s0]; a.auxZ = z->auxZ[s0];
    a.oauxR = z->auxR[s1]; a.oauxZ = z->auxZ[s1];
    a.mauxR = z->mauxR; a.mauxZ = z->mauxZ;
    a.m2auxR = z->m2auxR; a.m2auxZ = z->m2auxZ;
    a.rows = z->rows; a.zrows = z->zrows;
    a.k_mon = d.k_mon;
    a.k0 = d.design_k0; a.k1 = d.design_k1;
    a.kchunk = z->kchunk;
    a.tile_rows = z->tile_rows;
    a.xcd_remap = z->xcd_remap;
    a.nt_stores = z->nt_stores;
    return a;
}

zda_status reset_state(zda_zone *z, hipStream_t s)
{
    for (int b = 0; b < 2; ++b) {
        for (auto f : z->F[b]) if (f) launch_fill(f, z->ncell, s);
        if (z->auxR[b]) launch_fill(z->auxR[b], (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi, s);
        if (z->auxZ[b]) launch_fill(z->auxZ[b], (size_t)N_AUX_Z * z->dZ * z->plane, s);
    }
    if (z->mauxR) launch_fill(z->mauxR, (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi, s);
    if (z->mauxZ) launch_fill(z->mauxZ, (size_t)N_AUX_Z * z->dZ * z->plane, s);
    if (z->m2auxR) launch_fill(z->m2auxR, (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi, s);
    if (z->m2auxZ) launch_fill(z->m2auxZ, (size_t)N_AUX_Z * z->dZ * z->plane, s);
    if (z->flag) launch_set_int(z->flag, 0, s);
    z->cur = 0;
    HIP_TRY(hipGetLastError());
    z->n_done = 0;
    return ZDA_OK;
}

// The pulse of the source presets and of the adjoint mixing (window [0, 2 n0]).
double pulse_at(long n, double dt, double wc, double w, int n0)
{
    if (n < 0 || n > 2L * n0) return 0.0;
    const double t = (double)(n - n0) * dt;
    return std::sin(wc * t) * std::exp(-t * t / (2.0 * w * w));
}

int default_n0(double w, double dt) { return (int)std::lround(6.0 * w / dt); }

// Upload one run's source profiles and DFT twiddles (after the reset, if
// asked) and fill the step arguments of the two buffer parities (ab[0] = the
// zone's current set).  P source patterns are already on the device at
// rb.pattern; prof[p * nsteps + n] are the host complex profiles.
zda_status prepare_run(zda_zone *z, int m, int nsteps, int k_src, int P, const cd *prof, const double *omega, int K,
                       float2 *dft_plane, float2 *dft_vol, bool reset, hipStream_t s, StepArgs ab[2],
                       const RunBufs &rb)
{
    if (z->released) return released_error();
    // next to the axis the z components there are single-valued scalars; they
    // vanish (and the scheme holds) only when the seam phase is not 1
    if (z->d.axis && (z->d.n_fold > 0 ? m % z->d.n_fold == 0 : m == 0))
        return fail(ZDA_ERR_UNSUPPORTED, "axis zone with seam phase 1 (m = %d): the axis scalars do not vanish", m);
    const size_t T = (size_t)std::max(nsteps, 1);
    const size_t nprof = T * std::max(P, 1), ntw = T * std::max(K, 1);
    zda_status st;
    float2 *dprof = rb.profile, *dtw = rb.twiddle;
    if (rb.noalloc) {
        if (nprof > rb.cap_profile || ntw > rb.cap_twiddle) return fail(ZDA_ERR_ARG, "scratch slices too small");
    } else {
        if ((st = ensure(z, &z->profile, &z->cap_profile, nprof)) != ZDA_OK) return st;
        if ((st = ensure(z, &z->twiddle, &z->cap_twiddle, ntw)) != ZDA_OK) return st;
        dprof = z->profile;
        dtw = z->twiddle;
    }
    if (reset) {
        if ((st = reset_state(z, s)) != ZDA_OK) return st;
        if (dft_plane) launch_fill(dft_plane, (size_t)K * 2 * z->plane, s);
        if (dft_vol) launch_fill(dft_vol, (size_t)K * 3 * z->nd * z->plane, s);
    }
    float2 *hp = nullptr;
    if (rb.noalloc) {
        z->st_prof.assign(nprof + ntw, make_float2(0.f, 0.f));
        hp = z->st_prof.data();
    } else {
        hp = (float2 *)z->stage.take((nprof + ntw) * sizeof(float2));
        if (!hp) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
        std::memset((void *)hp, 0, (nprof + ntw) * sizeof(float2));
    }
    for (int n = 0; n < nsteps; ++n)
        for (int p = 0; p < P; ++p) {
            const cd g = prof[(size_t)p * nsteps + n];
            hp[(size_t)n * P + p] = make_float2((float)g.real(), (float)g.imag());
        }
    float2 *htw = hp + nprof;
    for (int n = 0; n < nsteps; ++n)
        for (int k = 0; k < K; ++k) {
            const double N = (double)(z->n_done + n + 1);
            const cd tw = z->dt * std::exp(cd(0.0, omega[k] * N * z->dt));
            htw[(size_t)n * K + k] = make_float2((float)tw.real(), (float)tw.imag());
        }
    HIP_TRY(hipMemcpyAsync(dprof, hp, nprof * sizeof(float2), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dtw, htw, ntw * sizeof(float2), hipMemcpyHostToDevice, s));
    if (!rb.noalloc) HIP_TRY(z->stage.issued(s));
    for (int b = 0; b < 2; ++b) {
        ab[b] = step_args(z, m);
        ab[b].k_src = k_src;
        ab[b].n_prof = P;
        ab[b].pattern = rb.pattern;
        ab[b].profile = dprof;
        ab[b].K = K;
        ab[b].twiddle = dtw;
        ab[b].dft_plane = dft_plane;
        ab[b].dft_vol = dft_vol;
        z->cur ^= 1;
    }
    return ZDA_OK;
}

// [lo, hi) cut into near-equal pieces of at most len
void split_range(int lo, int hi, int len, std::vector<std::pair<int, int>> &out)
{
    if (hi <= lo) return;
    const long L = hi - lo, q = (L + len - 1) / len;
    for (long p = 0; p < q; ++p) out.push_back({lo + (int)(L * p / q), lo + (int)(L * (p + 1) / q)});
}

// Tiles of the two-step kernel for one zone (TR rows, kc planes).  A tile
// computes rows i0-2 .. i0+nrow and planes kb-2 .. ke; it runs the
// instantiation without layer recursions when none of those rows and planes
// is a layer cell, i.e. when its rows lie in [pr0+2, nr-pr1-1) and its planes
// in [pz0+2, nz-pz1-1) (or reach an edge without a layer).  The layer bands
// are cut separately so that the layer-tile launch covers little more than
// the layers.  The fourth word of each descriptor is `tag` (the zone's index
// in a batch).
struct TwoStepTiles {
    // by the layer recursions a tile runs: [0] none, [1] the r- and z-layer
    // recursions with the auxiliaries carried in registers (TWO_CARRY_ROWS
    // owned rows), [2] the z-layer recursions only (tiles whose computed rows
    // hold no r-layer cell: the flat-mapped kernel, or carried in registers),
    // [3] the r- and z-layer recursions through the intermediate set
    std::vector<uint4> v[N_LAY];
    size_t cells = 0, mon = 0, src = 0;   // owned by the interior tiles
};

// Order code of a zone's two-step tile list: 0 natural (plane chunk, row
// band, phi column), 1 contiguous range per XCD, otherwise a patch shape
// (bands << 8) | columns.
int tile_order(const zda_zone *z)
{
    return z->tile_patch ? z->tile_patch : (z->xcd_remap ? 1 : 0);
}

void two_step_tiles(const zda_zone *z, int TR, int kc, int k_src, int order, unsigned tag, TwoStepTiles &t,
                    bool split_z = false, bool carry = false, bool three = false)
{
    // carry: the r-layer bands are cut into tiles of TWO_CARRY_ROWS rows for
    // the carrying instantiation, and the z-only tiles get their own launch.
    // three: the three-step kernel's tiles (interior rows in bands of TR,
    // r-layer bands in THREE_LAYER_ROWS, z-only tiles in their own launch),
    // whose computed rows and planes reach one further below and above
    if (split_z || three) carry = false;
    const int TRr = three ? THREE_LAYER_ROWS : carry ? TWO_CARRY_ROWS : TR;
    const int lo = three ? 3 : 2, hi = three ? 2 : 1;   // computed rows (planes) below and above a tile's own
    const zda_zone_desc &d = z->d;
    const int rA = d.pml_r_in > 0 ? std::min(d.pml_r_in + lo, d.nr) : 0;
    const int rB = d.pml_r_out > 0 ? std::max(d.nr - d.pml_r_out - hi, rA) : d.nr;
    const int zA = d.pml_z_lo > 0 ? std::min(d.pml_z_lo + lo, d.nz) : 0;
    const int zB = d.pml_z_hi > 0 ? std::max(d.nz - d.pml_z_hi - hi, zA) : d.nz;
    auto cols_of = [three](int lay) { return three ? three_step_cols(lay) : two_step_cols(lay); };
    std::vector<std::pair<int, int>> rows, rows2, planes;
    split_range(0, rA, TRr, rows);
    const size_t r_in0 = rows.size();
    split_range(rA, rB, TR, rows);
    const size_t r_in1 = rows.size();
    split_range(rB, d.nr, TRr, rows);
    // with carried auxiliaries, the chunks without z-layer planes cut an
    // r-layer band into TWO_RBAND_ROWS-row tiles of the r-layer-only
    // instantiation (lay 4) where that takes fewer wavefront rows than
    // TWO_CARRY_ROWS-row tiles: the 14- and 13-row bands of the 512 x 1024 x
    // 400 zone (layer launches 1.757 -> 1.597 ms), not the 10- and 9-row bands
    // of the 256 x 512 x 300 zone (0.462 -> 0.502 ms with 7-row tiles there)
    auto rband_rows = [&](int h) {
        if (!carry || h <= 0) return TRr;
        const int w7 = (h + TWO_RBAND_ROWS - 1) / TWO_RBAND_ROWS * (TWO_RBAND_ROWS + 3);
        const int w5 = (h + TWO_CARRY_ROWS - 1) / TWO_CARRY_ROWS * (TWO_CARRY_ROWS + 3);
        return w7 < w5 ? TWO_RBAND_ROWS : TRr;
    };
    const int TRq0 = rband_rows(rA), TRq1 = rband_rows(d.nr - rB);
    split_range(0, rA, TRq0, rows2);
    const size_t r2_in0 = rows2.size();
    split_range(rA, rB, TR, rows2);
    const size_t r2_in1 = rows2.size();
    split_range(rB, d.nr, TRq1, rows2);
    split_range(0, zA, kc, planes);
    const size_t z_in0 = planes.size();
    split_range(zA, zB, kc, planes);
    const size_t z_in1 = planes.size();
    split_range(zB, d.nz, kc, planes);
    auto gx_of = [&](int lay) { return (d.nphi + cols_of(lay) - 1) / cols_of(lay); };
    // chunk depth of the r-layer band tiles: given, or at most 48 (24 for
    // the tiles that carry their auxiliaries in registers) and halved (down
    // to 12 planes) while the layer launch would hold fewer than 512 tiles
    // (two blocks per CU).  With carried auxiliaries 24 planes measured best
    // of 8-96 on the 512 x 1024 x 400 zone (layer launches 1.772 -> 1.748
    // ms against 48) and on the 256 x 512 x 300 zone (0.564 -> 0.464 ms)
    int lkc = z->layer_kchunk > 0 ? std::min(z->layer_kchunk, kc) : std::min(kc, carry ? 24 : 48);
    if (z->layer_kchunk < 0) {
        const size_t r_bands = r2_in0 + (rows2.size() - r2_in1), z_chunks = z_in0 + (planes.size() - z_in1);
        const size_t z_tiles = z_chunks * (r_in1 - r_in0) * (size_t)gx_of(3);
        const size_t in_planes = (size_t)(z_in1 > z_in0 ? planes[z_in1 - 1].second - planes[z_in0].first : 0);
        auto layer_tiles = [&](int c) {
            return z_tiles + r_bands * (size_t)gx_of(3) * (z_chunks + (in_planes + c - 1) / c);
        };
        while (r_bands > 0 && lkc / 2 >= 12 && layer_tiles(lkc) < 512) lkc /= 2;
    }
    std::vector<uint4> v[N_LAY];
    for (size_t pz = 0; pz < planes.size(); ++pz) {
        const int kb = planes[pz].first, ke = planes[pz].second;
        const bool zl = !(pz >= z_in0 && pz < z_in1);
        const auto &R = zl ? rows : rows2;
        const size_t a0 = zl ? r_in0 : r2_in0, a1 = zl ? r_in1 : r2_in1;
        for (size_t pr = 0; pr < R.size(); ++pr) {
            const int i0 = R[pr].first, nrow = R[pr].second - R[pr].first;
            const bool rl = !(pr >= a0 && pr < a1);
            // without carried auxiliaries every tile with layer cells goes
            // to one launch of the full instantiation (lay 3): separate
            // launches for the z-only and r-only tiles measured slower there
            // on the 512 x 1024 x 400 zone, their partly filled last rounds
            // outweighing the gain.  With carried auxiliaries the r-layer
            // band tiles (lay 1, lay 4 as above) and the z-only tiles (lay 2)
            // take one launch each; so do the z-only tiles with split_z (the
            // flat-mapped kernel, whose lens batches hold many small tiles:
            // 2 % faster on the 16-zone LWIR-shaped lens)
            const int band_rows = pr < a0 ? TRq0 : TRq1;
            const int lay = rl ? (carry ? (!zl && band_rows == TWO_RBAND_ROWS ? 4 : 1) : 3)
                               : (zl ? (split_z || carry || three ? 2 : 3) : 0);
            const int cw = cols_of(lay);
            // r-layer band tiles carry ten recursions per cell: where they
            // are few, shorter chunks spread them over more blocks
            std::vector<std::pair<int, int>> sub;
            if (rl && !zl && lkc < kc) split_range(kb, ke, lkc, sub);
            else sub.push_back({kb, ke});
            for (const auto &sk : sub)
                for (int bx = 0; bx < gx_of(lay); ++bx) {
                    v[lay].push_back(make_uint4((unsigned)bx, (unsigned)i0 | ((unsigned)nrow << 16),
                                                (unsigned)sk.first | ((unsigned)sk.second << 16), tag));
                    if (lay == 0) {
                        const int j0 = bx * cw;
                        const size_t cols = (size_t)(std::min(j0 + cw, d.nphi) - j0);
                        t.cells += (size_t)nrow * cols * (size_t)(ke - kb);
                        if (d.k_mon >= kb && d.k_mon < ke) t.mon += (size_t)nrow * cols;
                        if (k_src >= kb && k_src < ke) t.src += (size_t)nrow * cols;
                    }
                }
        }
    }
    // with ZDA_OPT_XCD_REMAP, each of the eight XCDs (which take the blocks
    // of a launch round-robin) sweeps one contiguous range of the list, so
    // tiles that share halo rows and columns meet in one L2
    auto xcd_order = [](std::vector<uint4> &u) {
        const size_t nb = u.size();
        if (nb < 8) return;
        std::vector<uint4> o(nb);
        const size_t per = nb / 8, rem = nb % 8;
        size_t b = 0;
        for (size_t s = 0; b < nb; ++s)
            for (size_t x = 0; x < 8 && b < nb; ++x) {
                const size_t len = per + (x < rem ? 1 : 0);
                if (s < len) o[b++] = u[x * per + std::min(x, rem) + s];
            }
        u.swap(o);
    };
    // patch order: within each plane chunk, the (row band x phi column) grid
    // is cut into patches of PA bands x at most PB columns; patch q goes to
    // XCD q mod 8, which works through its patches in turn, so the tiles that
    // one XCD holds at a time are 2-D neighbours and share their halo lines in
    // its L2, while the eight XCDs together still sweep one compact region
    auto patch_order = [](std::vector<uint4> &u, int gx, int PA, int PB) {
        if (u.size() < 8) return;
        std::vector<std::pair<int, int>> cgs;
        split_range(0, gx, std::max(PB, 1), cgs);
        std::vector<std::vector<uint4>> seq(8);
        size_t q = 0, a = 0;
        while (a < u.size()) {                       // one plane chunk: tiles [a, b)
            size_t b = a;
            while (b < u.size() && u[b].z == u[a].z) ++b;
            std::vector<size_t> band;                // first tile of each row band
            for (size_t c = a; c < b; ++c)
                if (c == a || u[c].y != u[c - 1].y) band.push_back(c);
            band.push_back(b);
            for (size_t g = 0; g + 1 < band.size(); g += (size_t)std::max(PA, 1)) {
                const size_t g1 = std::min(g + (size_t)std::max(PA, 1), band.size() - 1);
                for (const auto &cg : cgs) {
                    std::vector<uint4> &s = seq[q++ % 8];
                    for (size_t bb = g; bb < g1; ++bb)
                        for (size_t c = band[bb]; c < band[bb + 1]; ++c)
                            if ((int)u[c].x >= cg.first && (int)u[c].x < cg.second) s.push_back(u[c]);
                }
            }
            a = b;
        }
        std::vector<uint4> o;
        o.reserve(u.size());
        for (size_t s = 0; o.size() < u.size(); ++s)
            for (int x = 0; x < 8; ++x)
                if (s < seq[x].size()) o.push_back(seq[x][s]);
        u.swap(o);
    };
    for (int q = 0; q < N_LAY; ++q) {
        if (order == 1) xcd_order(v[q]);
        else if (order > 1) patch_order(v[q], gx_of(q), order >> 8, order & 0xff);
        t.v[q].insert(t.v[q].end(), v[q].begin(), v[q].end());
    }
}

// Default chunk depth of the two-step interior tiles: the candidate whose
// launch finishes first if every tile takes time in proportion to the planes
// it computes (its chunk plus three) and the tiles run in rounds of one per
// CU: ceil(tiles / n_cu) x (chunk + 3); a tie keeps the shallower candidate
// (deeper candidates that cut the planes into the same chunks tie).  It picks
// 72 planes on the 256 x 512 x 300 zone (measured 3.4 % faster per step than
// 48; 40 planes, the runner-up, 5.6 %), 64 on the 512 x 1024 x 400 zone (1 %)
// and 3 on the 64 x 64 x 96 zone, whose tiles fit in one round (forward +
// adjoint iteration 0.38 -> 0.26 s).
int default_two_step_kchunk(const zda_zone_desc &d, int n_cu)
{
    const int rA = d.pml_r_in > 0 ? std::min(d.pml_r_in + 2, d.nr) : 0;
    const int rB = d.pml_r_out > 0 ? std::max(d.nr - d.pml_r_out - 1, rA) : d.nr;
    const int zA = d.pml_z_lo > 0 ? std::min(d.pml_z_lo + 2, d.nz) : 0;
    const int zB = d.pml_z_hi > 0 ? std::max(d.nz - d.pml_z_hi - 1, zA) : d.nz;
    const long bands = (rB - rA + 12) / 13, gx = (d.nphi + two_step_cols(0) - 1) / two_step_cols(0);
    const long planes = std::max(zB - zA, 1);
    int best = std::min(3, d.nz);
    double best_cost = 1e300;
    for (int kc : {3, 4, 6, 8, 12, 16, 24, 32, 40, 48, 56, 64, 72}) {
        if (kc > d.nz) break;
        const long chunks = (planes + kc - 1) / kc;
        const long len = (planes + chunks - 1) / chunks;
        const long tiles = std::max(bands * gx * chunks, 1L);
        const double cost = (double)((tiles + n_cu - 1) / n_cu) * (double)(len + 3);
        if (cost < best_cost) { best_cost = cost; best = kc; }
    }
    return best;
}

// Owned rows of a two-step tile for a tile_rows code (the code itself, or
// the rows a flat block holds less its halo)
int two_step_rows(int tile_rows, int nphi)
{
    return tile_rows == FLAT_TWO_ROWS ? flat_two_rows(nphi) : tile_rows;
}

// A zone's two-step tile list (interior tiles first) and its counts.
void plan_zone_tiles(const zda_zone *z, std::vector<uint4> &all, TileCounts &tc)
{
    const int TR = z->tile_rows;
    TwoStepTiles t;
    two_step_tiles(z, two_step_rows(TR, z->d.nphi), z->kchunk, z->k_src_last, tile_order(z), 0u, t,
                   TR == FLAT_TWO_ROWS, z->layer_carry != 0, z->three);
    all.clear();
    for (int q = 0; q < N_LAY; ++q) {
        tc.n_lay[q] = (unsigned)t.v[q].size();
        all.insert(all.end(), t.v[q].begin(), t.v[q].end());
    }
    tc.cells = t.cells;
    tc.mon = t.mon;
    tc.src = t.src;
}

// The zone's own tile list, rebuilt when the launch shape, the source plane
// or the tile order changed.
zda_status build_two_step_tiles(zda_zone *z, hipStream_t s)
{
    const int TR = z->tile_rows, kc = z->kchunk;
    if (z->tiles2 && z->tiles_tr == TR && z->tiles_kc == kc && z->tiles_src == z->k_src_last &&
        z->tiles_xcd == tile_order(z) && z->tiles_lkc == z->layer_kchunk && z->tiles_carry == z->layer_carry)
        return ZDA_OK;
    std::vector<uint4> all;
    TileCounts tc;
    plan_zone_tiles(z, all, tc);
    zda_status st = ensure(z, &z->tiles2, &z->cap_tiles2, all.size());
    if (st != ZDA_OK) return st;
    void *h = z->stage.take(all.size() * sizeof(uint4));
    if (!h) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
    std::memcpy(h, all.data(), all.size() * sizeof(uint4));
    HIP_TRY(hipMemcpyAsync(z->tiles2, h, all.size() * sizeof(uint4), hipMemcpyHostToDevice, s));
    HIP_TRY(z->stage.issued(s));
    z->tc = tc;
    z->tiles_src = z->k_src_last;
    z->tiles_tr = TR;
    z->tiles_kc = kc;
    z->tiles_xcd = tile_order(z);
    z->tiles_lkc = z->layer_kchunk;
    z->tiles_carry = z->layer_carry;
    return ZDA_OK;
}

// In-loop divergence check of the zone's newest fields
void watch_fields(zda_zone *z, hipStream_t s)
{
    WatchArgs w{};
    for (int c = 0; c < 6; ++c) w.f[c] = z->F[z->cur][c];
    w.n = z->ncell;
    w.flag = z->flag;
    w.bound2 = WATCH_BOUND2;
    launch_watch(w, s);
}

// rb: where the run's inputs are staged (rb.tiles / rb_tc: the two-step tile
// list of the entry point that allocates nothing; otherwise the zone's own)
zda_status run_loop(zda_zone *z, int m, int nsteps, int k_src, int P, const cd *prof, const double *omega, int K,
                    float2 *dft_plane, float2 *dft_vol, bool reset, hipStream_t s, const RunBufs &rb,
                    bool timing = false, const TileCounts *rb_tc = nullptr)
{
    StepArgs ab[2];
    zda_status st = prepare_run(z, m, nsteps, k_src, P, prof, omega, K, dft_plane, dft_vol, reset, s, ab, rb);
    if (st != ZDA_OK) return st;
    const int ab_base = z->cur;
    const StepArgs &a = ab[0];
    const bool fused = z->fused, two = z->two;
    // steps per launch of the multi-step kernels (the two-step family, or
    // the three-step kernel); a run's last nsteps mod depth steps take the
    // fused one-step kernel
    const int depth = z->three ? 3 : 2;
    z->k_src_last = k_src;
    const uint4 *tiles = nullptr;
    TileCounts tc;
    if (two) {
        if (rb.noalloc) {
            tiles = rb.tiles;
            tc = *rb_tc;
        } else {
            if ((st = build_two_step_tiles(z, s)) != ZDA_OK) return st;
            tiles = z->tiles2;
            tc = z->tc;
        }
    }
    unsigned n_pml = 0;
    for (int q = 1; q < N_LAY; ++q) n_pml += tc.n_lay[q];
    // in-loop divergence watchdog every watch_every steps of the zone's clock
    const long W = z->watch_every;
    long next_watch = W > 0 ? ((long)z->n_done / W + 1) * W : -1;
    auto watch = [&](int done) {
        if (W <= 0 || (long)z->n_done + done < next_watch) return;
        watch_fields(z, s);
        while (next_watch <= (long)z->n_done + done) next_watch += W;
    };
    // one step of the one-launch kernel (the fused step, or an odd last step
    // of a two-step run)
    auto one_step = [&](int n) {
        if (fused || two) {
            StepArgs b = ab[z->cur ^ ab_base];
            if (two) b.tile_rows = z->tile_rows == FLAT_TWO_ROWS ? FLAT_FUSED_ROWS : 3;
            launch_fused_step(b, n, s);
            z->cur ^= 1;
        } else {
            launch_h_step(a, n, s);
            launch_e_step(a, n, s);
        }
    };
    // steps n .. n + depth - 1 by the multi-step kernel; ev (if given)
    // brackets the interior-tile and the layer-tile launches
    const bool conc = two && z->layer_stream && n_pml > 0 && !rb.noalloc;
    if (conc && !z->s2) {
        HIP_TRY(hipStreamCreateWithFlags(&z->s2, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&z->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&z->ev_join, hipEventDisableTiming));
    }
    // the three layer-tile lists (r rows only, z planes only, both), each
    // with its own instantiation
    auto layer_launches = [&](StepArgs b, int n, hipStream_t st) {
        size_t off = tc.n_lay[0];
        for (int q = 1; q < N_LAY; ++q) {
            b.tiles = tiles + off;
            if (depth == 3) launch_three_step(b, n, tc.n_lay[q], q, st);
            else launch_two_step(b, n, tc.n_lay[q], q, st);
            off += tc.n_lay[q];
        }
    };
    auto two_steps = [&](int n, hipEvent_t *ev) -> zda_status {
        StepArgs b = ab[z->cur ^ ab_base];
        hipStream_t sl = s;
        if (conc) {   // layer tiles on the zone's second stream, forked from and joined into s
            HIP_TRY(hipEventRecord(z->ev_fork, s));
            HIP_TRY(hipStreamWaitEvent(z->s2, z->ev_fork, 0));
            sl = z->s2;
            if (ev) HIP_TRY(hipEventRecord(ev[2], sl));
            layer_launches(b, n, sl);
            if (ev) HIP_TRY(hipEventRecord(ev[3], sl));
        }
        b.tiles = tiles;
        if (ev) HIP_TRY(hipEventRecord(ev[0], s));
        if (depth == 3) launch_three_step(b, n, tc.n_lay[0], 0, s);
        else launch_two_step(b, n, tc.n_lay[0], 0, s);
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
        if (conc) {
            HIP_TRY(hipEventRecord(z->ev_join, sl));
            HIP_TRY(hipStreamWaitEvent(s, z->ev_join, 0));
        } else {
            if (ev) HIP_TRY(hipEventRecord(ev[2], s));
            layer_launches(b, n, s);
            if (ev) HIP_TRY(hipEventRecord(ev[3], s));
        }
        z->cur ^= 1;
        return ZDA_OK;
    };
    z->timed_steps = 0;
    if (timing) {
        const size_t need = 4 * (size_t)nsteps;
        while (z->ev.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            z->ev.push_back(e);
        }
        int groups = 0;
        if (two) {
            int n = 0;
            for (; n + depth - 1 < nsteps; n += depth, ++groups) {
                if ((st = two_steps(n, &z->ev[4 * (size_t)groups])) != ZDA_OK) return st;
                watch(n + depth);
            }
            for (; n < nsteps; ++n) {
                one_step(n);
                watch(n + 1);
            }
        } else {
            for (int n = 0; n < nsteps; ++n, ++groups) {
                if (fused) {
                    HIP_TRY(hipEventRecord(z->ev[4 * n + 2], s));
                    one_step(n);
                    HIP_TRY(hipEventRecord(z->ev[4 * n + 3], s));
                } else {
                    HIP_TRY(hipEventRecord(z->ev[4 * n], s));
                    launch_h_step(a, n, s);
                    HIP_TRY(hipEventRecord(z->ev[4 * n + 1], s));
                    HIP_TRY(hipEventRecord(z->ev[4 * n + 2], s));
                    launch_e_step(a, n, s);
                    HIP_TRY(hipEventRecord(z->ev[4 * n + 3], s));
                }
                watch(n + 1);
            }
        }
        z->timed_steps = groups;
        z->timed_fused = fused || two;
        z->timed_two = two;
        z->timed_depth = depth;
        z->timed_tc = tc;
    } else if (two) {
        int n = 0;
        for (; n + depth - 1 < nsteps; n += depth) {
            if ((st = two_steps(n, nullptr)) != ZDA_OK) return st;
            watch(n + depth);
        }
        for (; n < nsteps; ++n) {
            one_step(n);
            watch(n + 1);
        }
    } else {
        for (int n = 0; n < nsteps; ++n) {
            one_step(n);
            watch(n + 1);
        }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(post_flag(z, s));
    z->n_done += nsteps;
    return ZDA_OK;
}


// Forward-run setup shared by the single-zone and batched runs: argument
// checks, source pattern and profiles, DFT buffers.
struct FwdPlan {
    int P = 1;
    std::vector<cd> prof;
    double width = 0.0;
    int n0 = -1;
    float2 *dplane = nullptr, *dvol = nullptr;
    bool reset = true;
};

// The plane-wave sheet of the presets on the host: J_r = -e^{i m phi_j}/dz,
// J_phi = -i sgn(m) e^{i m phi_{j+1/2}}/dz (|m| = 1), or J_r = -1/dz (radial,
// m = 0); the pulse multiplies it.  out: [2][nr][nphi].
template <typename V>
void preset_pattern_host(const zda_zone *z, int kind, V *out)
{
    using R = decltype(out->x);
    const zda_zone_desc &d = z->d;
    const double sgn = d.m > 0 ? 1.0 : (d.m < 0 ? -1.0 : 0.0);
    for (int i = 0; i < d.nr; ++i)
        for (int j = 0; j < d.nphi; ++j) {
            cd jr, jp;
            if (kind == ZDA_SRC_PLANE_CIRC) {
                // sample points phi_j, phi_{j+1/2} (all at phi = 0 in a continuous zone)
                const double pj = d.n_fold > 0 ? j * z->dphi : 0.0;
                const double ph = d.n_fold > 0 ? (j + 0.5) * z->dphi : 0.0;
                jr = -std::exp(cd(0.0, d.m * pj)) / d.dz;
                jp = cd(0.0, -sgn) * std::exp(cd(0.0, d.m * ph)) / d.dz;
            } else {
                jr = -1.0 / d.dz;
                jp = 0.0;
            }
            V &a = out[(size_t)i * d.nphi + j], &b = out[z->plane + (size_t)i * d.nphi + j];
            a.x = (R)jr.real();
            a.y = (R)jr.imag();
            b.x = (R)jp.real();
            b.y = (R)jp.imag();
        }
}

// Patterns a source needs on the device (1 for the presets).
int source_patterns(const zda_source *s) { return s->kind == ZDA_SRC_CUSTOM ? s->n_profiles : 1; }

zda_status forward_setup(zda_zone *z, const zda_source *s, int nsteps, const double *omega, int K, int dft_flags,
                         hipStream_t hs, FwdPlan &plan, RunBufs &rb)
{
    if (nsteps < 0) return fail(ZDA_ERR_ARG, "nsteps must be >= 0");
    if (K < 0 || K > ZDA_MAX_FREQ || (K > 0 && !omega)) return fail(ZDA_ERR_ARG, "K must be in [0, %d]", ZDA_MAX_FREQ);
    if ((dft_flags & ~(ZDA_DFT_PLANE | ZDA_DFT_VOLUME | ZDA_RUN_CONTINUE | ZDA_RUN_TIMING)) != 0)
        return fail(ZDA_ERR_ARG, "bad dft_flags");
    if ((dft_flags & ZDA_DFT_VOLUME) && z->nd <= 0) return fail(ZDA_ERR_STATE, "zone has no design layer");
    const zda_zone_desc &d = z->d;
    if (s->k_src < 1 || s->k_src >= d.nz) return fail(ZDA_ERR_ARG, "k_src must be in [1, nz)");
    plan.reset = !(dft_flags & ZDA_RUN_CONTINUE);
    if (plan.reset) z->n_done = 0;
    zda_status st;
    if (s->kind == ZDA_SRC_PLANE_CIRC || s->kind == ZDA_SRC_RADIAL) {
        if (s->kind == ZDA_SRC_PLANE_CIRC && std::abs(d.m) != 1) return fail(ZDA_ERR_UNSUPPORTED, "PLANE_CIRC needs |m| = 1");
        if (s->kind == ZDA_SRC_RADIAL && d.m != 0) return fail(ZDA_ERR_UNSUPPORTED, "RADIAL needs m = 0");
        if (!(s->width > 0)) return fail(ZDA_ERR_ARG, "pulse width must be > 0");
        plan.P = 1;
        plan.width = s->width;
        plan.n0 = s->n0 >= 0 ? s->n0 : default_n0(plan.width, z->dt);
        const size_t bytes = 2 * z->plane * sizeof(float2);
        if (rb.noalloc) {
            if (2 * z->plane > rb.cap_pattern) return fail(ZDA_ERR_ARG, "scratch slice too small for the pattern");
            z->st_pat.resize(2 * z->plane);
            preset_pattern_host(z, s->kind, z->st_pat.data());
            HIP_TRY(hipMemcpyAsync(rb.pattern, z->st_pat.data(), bytes, hipMemcpyHostToDevice, hs));
        } else {
            if ((st = ensure(z, &z->pattern, &z->cap_pattern, 2 * z->plane)) != ZDA_OK) return st;
            // the sheet depends only on the zone and the preset: rebuilt and
            // uploaded when the pattern buffer holds something else
            const int key = 1 + s->kind;
            if (z->pattern_key != key) {
                float2 *h = (float2 *)z->stage.take(bytes);
                if (!h) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
                preset_pattern_host(z, s->kind, h);
                HIP_TRY(hipMemcpyAsync(z->pattern, h, bytes, hipMemcpyHostToDevice, hs));
                HIP_TRY(z->stage.issued(hs));
                z->pattern_key = key;
            }
            rb.pattern = z->pattern;
        }
        plan.prof.resize(nsteps);
        for (int n = 0; n < nsteps; ++n) plan.prof[n] = pulse_at(z->n_done + n, z->dt, s->omega_c, plan.width, plan.n0);
    } else if (s->kind == ZDA_SRC_CUSTOM) {
        plan.P = s->n_profiles;
        if (plan.P < 1 || plan.P > ZDA_MAX_FREQ || !s->patterns || !s->profiles)
            return fail(ZDA_ERR_ARG, "CUSTOM needs 1..%d patterns and profiles", ZDA_MAX_FREQ);
        const size_t count = (size_t)plan.P * 2 * z->plane, bytes = count * sizeof(float2);
        float2 *dst = rb.pattern;
        if (rb.noalloc) {
            if (count > rb.cap_pattern) return fail(ZDA_ERR_ARG, "scratch slice too small for the patterns");
        } else {
            if ((st = ensure(z, &z->pattern, &z->cap_pattern, count)) != ZDA_OK) return st;
            dst = rb.pattern = z->pattern;
            z->pattern_key = 0;
        }
        if (s->patterns_on_device) {
            HIP_TRY(hipMemcpyAsync(dst, s->patterns, bytes, hipMemcpyDeviceToDevice, hs));
        } else if (rb.noalloc) {
            z->st_pat.resize(count);
            std::memcpy((void *)z->st_pat.data(), s->patterns, bytes);
            HIP_TRY(hipMemcpyAsync(dst, z->st_pat.data(), bytes, hipMemcpyHostToDevice, hs));
        } else {
            void *h = z->stage.take(bytes);
            if (!h) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
            std::memcpy(h, s->patterns, bytes);
            HIP_TRY(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, hs));
            HIP_TRY(z->stage.issued(hs));
        }
        plan.prof.resize((size_t)plan.P * nsteps);
        for (size_t q = 0; q < plan.prof.size(); ++q) plan.prof[q] = cd(s->profiles[2 * q], s->profiles[2 * q + 1]);
    } else {
        return fail(ZDA_ERR_ARG, "unknown source kind %d", s->kind);
    }
    plan.dplane = (dft_flags & ZDA_DFT_PLANE) && K > 0 ? z->dft_plane : nullptr;
    plan.dvol = nullptr;
    if ((dft_flags & ZDA_DFT_VOLUME) && K > 0) {
        if (!z->dft_vol) {
            if (rb.noalloc)
                return fail(ZDA_ERR_STATE, "the design-layer DFT buffer is allocated by a first zda_fdtd_run with "
                                           "ZDA_DFT_VOLUME");
            if ((st = dev_alloc(z, &z->dft_vol, (size_t)ZDA_MAX_FREQ * 3 * z->nd * z->plane)) != ZDA_OK) return st;
            launch_fill(z->dft_vol, (size_t)ZDA_MAX_FREQ * 3 * z->nd * z->plane, hs);
        }
        plan.dvol = z->dft_vol;
    }
    return ZDA_OK;
}

void forward_finish(zda_zone *z, const FwdPlan &plan, int nsteps, const double *omega, int K)
{
    if (plan.reset) {
        z->last_K = K;
        for (int k = 0; k < K; ++k) z->last_omega[k] = omega[k];
        z->last_T = nsteps;
        z->have_plane = plan.dplane != nullptr;
        z->have_vol = plan.dvol != nullptr;
    } else {
        // continuing: the monitors keep accumulating from the current state
        z->last_T += nsteps;
        if (plan.dplane || plan.dvol) {
            z->last_K = K;
            for (int k = 0; k < K; ++k) z->last_omega[k] = omega[k];
        }
        if (plan.dplane) z->have_plane = true;
        if (plan.dvol) z->have_vol = true;
    }
    z->last_width = plan.width;
    z->last_n0 = plan.n0;
    z->have_vol_adj = false;
}

// Gauss-Jordan inverse of a small complex matrix (row-major, n x n).
bool invert(std::vector<cd> &A, int n)
{
    std::vector<cd> inv(n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(A[r * n + c]) > std::abs(A[piv * n + c])) piv = r;
        if (std::abs(A[piv * n + c]) == 0.0) return false;
        for (int q = 0; q < n; ++q) { std::swap(A[c * n + q], A[piv * n + q]); std::swap(inv[c * n + q], inv[piv * n + q]); }
        const cd p = A[c * n + c];
        for (int q = 0; q < n; ++q) { A[c * n + q] /= p; inv[c * n + q] /= p; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const cd f = A[r * n + c];
            for (int q = 0; q < n; ++q) { A[r * n + q] -= f * A[c * n + q]; inv[r * n + q] -= f * inv[c * n + q]; }
        }
    }
    A = inv;
    return true;
}

// Adjoint-run setup (a7): the current pattern W^{-1} dF/dEhat_k / (i wt_k)
// on the monitor plane (built on the GPU) and the broadband time profiles
// q_k = sum_l (P^{-1})_{lk} p_l; the overlap weights are uploaded for the
// finish step.
struct AdjPlan {
    std::vector<cd> q;
    int K = 0, T = 0;
    float2 *wr_dev = nullptr, *wz_dev = nullptr;
    float *gtmp = nullptr;         // the gradient before its copy into host memory
};

zda_status adjoint_setup(zda_zone *z, const float *dF_dE, int dF_on_device, double adj_width, hipStream_t hs,
                         AdjPlan &plan)
{
    if (!z->have_vol || z->last_K < 1) return fail(ZDA_ERR_STATE, "needs a forward run with ZDA_DFT_VOLUME");
    const zda_zone_desc &d = z->d;
    const int K = z->last_K, T = z->last_T, km = d.k_mon, nd = z->nd;
    double width = adj_width > 0 ? adj_width : z->last_width;
    if (!(width > 0)) return fail(ZDA_ERR_ARG, "adjoint pulse width unknown (custom forward source): pass adj_width");
    const int n0 = (adj_width > 0 || z->last_n0 < 0) ? default_n0(width, z->dt) : z->last_n0;
    zda_status st;
    const size_t npl = (size_t)K * 2 * z->plane;
    const size_t nfac = (size_t)K * 2 * d.nr, nwr = (size_t)K * 3 * d.nr, nwz = (size_t)K * 3 * nd;
    const size_t ngt = ((size_t)nd * z->plane + 1) / 2;   // FP32 gradient in float2 units
    if ((st = ensure(z, &z->scratch, &z->cap_scratch, npl + nfac + nwr + nwz + ngt)) != ZDA_OK) return st;
    if ((st = ensure(z, &z->pattern, &z->cap_pattern, npl)) != ZDA_OK) return st;
    z->pattern_key = 0;
    if (!z->dft_vol_adj && (st = dev_alloc(z, &z->dft_vol_adj, (size_t)ZDA_MAX_FREQ * 3 * nd * z->plane)) != ZDA_OK)
        return st;
    float2 *g_dev = z->scratch, *fac_dev = g_dev + npl, *wr_dev = fac_dev + nfac, *wz_dev = wr_dev + nwr;
    plan.gtmp = (float *)(wz_dev + nwz);
    if (dF_on_device) {
        HIP_TRY(hipMemcpyAsync(g_dev, dF_dE, npl * sizeof(float2), hipMemcpyDeviceToDevice, hs));
    } else {
        void *h = z->stage.take(npl * sizeof(float2));
        if (!h) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
        std::memcpy(h, dF_dE, npl * sizeof(float2));
        HIP_TRY(hipMemcpyAsync(g_dev, h, npl * sizeof(float2), hipMemcpyHostToDevice, hs));
        HIP_TRY(z->stage.issued(hs));
    }
    // stretched volume W = R l_r l_z dphi and leap-frog frequency wt
    auto wt = [&](double w) { return 2.0 / z->dt * std::sin(w * z->dt / 2.0); };
    auto w_r = [&](int comp, int i, double w) {   // comp 0 = E_r (half point), 1, 2 = E_phi, E_z (integer)
        const int h = comp == 0 ? 1 : 0;
        const double r = d.r_in + (i + 0.5 * h) * d.dr;
        return r * stretch(z->sgt_r[h][i], z->cr, w, z->dt) * stretch(z->sig_r[h][i], z->cr, w, z->dt) * d.dr *
               z->dphi * d.dz;
    };
    auto w_z = [&](int comp, int k, double w) {
        const int h = comp == 2 ? 1 : 0;
        return stretch(z->sig_z[h][k], z->cz, w, z->dt);
    };
    float2 *misc = (float2 *)z->stage.take((nfac + nwr + nwz) * sizeof(float2));
    if (!misc) return fail(ZDA_ERR_HIP, "pinned staging allocation failed");
    std::memset((void *)misc, 0, (nfac + nwr + nwz) * sizeof(float2));
    for (int k = 0; k < K; ++k) {
        const double w = z->last_omega[k];
        for (int a = 0; a < 2; ++a)
            for (int i = 0; i < d.nr; ++i) {
                const cd f = 1.0 / (w_r(a, i, w) * w_z(a, km, w) * cd(0.0, wt(w)));
                misc[((size_t)k * 2 + a) * d.nr + i] = make_float2((float)f.real(), (float)f.imag());
            }
        for (int a = 0; a < 3; ++a) {
            for (int i = 0; i < d.nr; ++i) {
                const cd v = wt(w) * wt(w) * w_r(a, i, w);
                misc[nfac + ((size_t)k * 3 + a) * d.nr + i] = make_float2((float)v.real(), (float)v.imag());
            }
            for (int kd = 0; kd < nd; ++kd) {
                const cd v = w_z(a, d.design_k0 + kd, w);
                misc[nfac + nwr + ((size_t)k * 3 + a) * nd + kd] = make_float2((float)v.real(), (float)v.imag());
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(fac_dev, misc, (nfac + nwr + nwz) * sizeof(float2), hipMemcpyHostToDevice, hs));
    HIP_TRY(z->stage.issued(hs));
    launch_adjoint_pattern(z->pattern, g_dev, fac_dev, K, d.nr, d.nphi, hs);
    // broadband profiles: pulses p_l centred on w_l, mixed by P^{-1}, P_kl = phat_l(w_k)
    std::vector<double> p((size_t)K * T);
    for (int l = 0; l < K; ++l)
        for (int n = 0; n < T; ++n) p[(size_t)l * T + n] = pulse_at(n, z->dt, z->last_omega[l], width, n0);
    std::vector<cd> Pm((size_t)K * K);
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            cd acc = 0.0;
            for (int n = 0; n < T; ++n)
                acc += p[(size_t)l * T + n] * std::exp(cd(0.0, z->last_omega[k] * (n + 0.5) * z->dt));
            Pm[(size_t)k * K + l] = z->dt * acc;
        }
    if (!invert(Pm, K)) return fail(ZDA_ERR_ARG, "adjoint pulse spectra are singular at the chosen frequencies");
    std::vector<cd> q((size_t)K * T, 0.0);
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            const cd c = Pm[(size_t)l * K + k];
            for (int n = 0; n < T; ++n) q[(size_t)k * T + n] += c * p[(size_t)l * T + n];
        }
    plan.q.swap(q);
    plan.K = K;
    plan.T = T;
    plan.wr_dev = wr_dev;
    plan.wz_dev = wz_dev;
    return ZDA_OK;
}

// a9: dF/drho = (eps_hi - eps_bg) sum_k sum_alpha 2 Re[wt^2 W Xhat Ehat]
zda_status adjoint_finish(zda_zone *z, const AdjPlan &plan, float *grad_rho, int grad_on_device, hipStream_t hs)
{
    const zda_zone_desc &d = z->d;
    const int nd = z->nd, K = plan.K;
    z->have_vol_adj = true;
    float *gdst = grad_on_device ? grad_rho : plan.gtmp;
    launch_overlap(gdst, z->dft_vol, z->dft_vol_adj, plan.wr_dev, plan.wz_dev, K, nd, d.nr, d.nphi,
                   (float)(2.0 * (d.eps_hi - d.eps_bg)), hs);
    HIP_TRY(hipGetLastError());
    if (!grad_on_device) {
        HIP_TRY(hipMemcpyAsync(grad_rho, plan.gtmp, (size_t)nd * z->plane * sizeof(float), hipMemcpyDeviceToHost, hs));
        HIP_TRY(post_flag(z, hs));
        HIP_TRY(hipStreamSynchronize(hs));
        if (*z->flag_host) return fail(ZDA_ERR_DIVERGED, "the watchdog found non-finite or exploding fields");
    }
    return ZDA_OK;
}

}  // namespace

extern "C" {

zda_status zda_set_allocator(zda_alloc_fn alloc_fn, zda_free_fn free_fn, void *ctx)
{
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return fail(ZDA_ERR_ARG, "give both allocator functions, or neither (hipMalloc / hipFree)");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_alloc.alloc = alloc_fn;
    g_alloc.free = free_fn;
    g_alloc.ctx = alloc_fn ? ctx : nullptr;
    return ZDA_OK;
}

void zda_zone_desc_default(zda_zone_desc *d)
{
    if (!d) return;
    std::memset(d, 0, sizeof *d);
    d->n_fold = 1;
    d->dr = d->dz = 1.0;
    d->courant = 0.5;
    d->pml_r_in = d->pml_r_out = d->pml_z_lo = d->pml_z_hi = 8;
    d->pml_order = 3.0;
    d->pml_alpha = 0.05;
    d->eps_bg = 1.0;
    d->eps_hi = 6.25;
}

zda_status zda_zone_create(const zda_zone_desc *d, const float *eps, int eps_on_device, zda_zone **out)
{
    if (!d || !out) return fail(ZDA_ERR_ARG, "NULL descriptor or output");
    *out = nullptr;
    if (d->nr < 1 || d->nphi < 1 || d->nz < 2 || d->n_fold < 0)
        return fail(ZDA_ERR_ARG, "sizes must be >= 1 (nz >= 2) and n_fold >= 0");
    if (d->n_fold == 0 && d->nphi != 1) return fail(ZDA_ERR_ARG, "a continuous zone (n_fold = 0) has nphi = 1");
    if (!(d->dr > 0) || !(d->dz > 0) || !(d->courant > 0)) return fail(ZDA_ERR_ARG, "dr, dz, courant must be > 0");
    if (!(d->r_in > 0)) return fail(ZDA_ERR_UNSUPPORTED, "r_in must be > 0 (an axis zone has r_in = dr / 2)");
    if (d->axis && (d->pml_r_in != 0 || std::abs(d->r_in - 0.5 * d->dr) > 1e-12 * d->dr))
        return fail(ZDA_ERR_ARG, "an axis zone has r_in = dr / 2 and no inner r-layer");
    if (d->pml_r_in < 0 || d->pml_r_out < 0 || d->pml_z_lo < 0 || d->pml_z_hi < 0 ||
        2 * d->pml_r_in > d->nr || 2 * d->pml_r_out > d->nr || 2 * d->pml_z_lo > d->nz || 2 * d->pml_z_hi > d->nz)
        return fail(ZDA_ERR_ARG, "PML widths must be in [0, extent/2]");
    if (d->k_mon < 1 || d->k_mon >= d->nz) return fail(ZDA_ERR_ARG, "k_mon must be in [1, nz)");
    if (!(d->design_k0 == 0 && d->design_k1 == 0) &&
        (d->design_k0 < 0 || d->design_k1 > d->nz || d->design_k0 >= d->design_k1))
        return fail(ZDA_ERR_ARG, "design layer must satisfy 0 <= k0 < k1 <= nz");
    if (!(d->pml_order > 0) || d->pml_alpha < 0) return fail(ZDA_ERR_ARG, "bad PML profile");
    // continuous zone: dphi = tau = 1 and the phi difference is exactly i m / r,
    // whose CFL term is (m / (2 r))^2 (a Yee direction contributes (1/h)^2)
    const double dphi = d->n_fold > 0 ? 2.0 * M_PI / ((double)d->n_fold * d->nphi) : 1.0;
    const double dt = d->courant * std::min(d->dr, d->dz);
    const double q = d->n_fold > 0 ? 1.0 / (d->r_in * dphi) : std::abs((double)d->m) / (2.0 * d->r_in);
    const double cfl = dt * std::sqrt(1.0 / (d->dr * d->dr) + q * q + 1.0 / (d->dz * d->dz));
    if (cfl >= 1.0) return fail(ZDA_ERR_CFL, "Courant number %.4f >= 1 (dt sqrt(1/dr^2+q^2+1/dz^2))", cfl);

    zda_zone *z = new (std::nothrow) zda_zone();
    if (!z) return fail(ZDA_ERR_OOM, "host allocation failed");
    z->d = *d;
    if (hipGetDevice(&z->device) != hipSuccess) { delete z; return fail(ZDA_ERR_HIP, "no HIP device"); }
    z->mem.al = current_allocator();
    z->mem.device = z->device;
    z->dphi = dphi;
    z->tau = d->n_fold > 0 ? 2.0 * M_PI / d->n_fold : 1.0;
    z->dt = dt;
    z->cfl = cfl;
    z->plane = (size_t)d->nr * d->nphi;
    z->ncell = z->plane * d->nz;
    z->dR = d->pml_r_in + d->pml_r_out;
    z->dZ = d->pml_z_lo + d->pml_z_hi;
    z->nd = d->design_k1 - d->design_k0;
    // default launch shape of the fused step (measured on the 512 x 1024 x
    // 400 zone): 3 owned rows per block, 12-plane z-chunks; shorter chunks
    // (down to 4 planes) while the grid has fewer than 2048 blocks.  Zones
    // with room for the intermediate auxiliaries switch to the two-step
    // kernel below.
    const bool narrow = d->nphi <= NARROW_PHI;
    {
        z->tile_rows = 3;
        const long tiles = (long)((d->nphi + FUSED_COLS - 1) / FUSED_COLS) * ((d->nr + 2) / 3);
        int kc = std::min(12, d->nz);
        while (kc > 4 && tiles * ((d->nz + kc - 1) / kc) < 2048) --kc;
        z->kchunk = kc;
    }
    std::vector<RowCoef> rows;
    std::vector<ZCoef> zr;
    setup_layers(z, rows, zr);

    zda_status st = ZDA_OK;
    for (auto &f : z->F[0]) if (st == ZDA_OK) st = dev_alloc(z, &f, z->ncell);
    if (st == ZDA_OK) st = dev_alloc(z, &z->ceps, z->ncell);
    if (st == ZDA_OK) st = dev_alloc(z, &z->auxR[0], (size_t)N_AUX_R * d->nz * z->dR * d->nphi);
    if (st == ZDA_OK) st = dev_alloc(z, &z->auxZ[0], (size_t)N_AUX_Z * z->dZ * z->plane);
    // the second buffer set of the fused step; without room for it (or when
    // asked for a single set) the zone keeps the in-place split kernels
    if (st == ZDA_OK && d->single_buffer) {
        z->fused = false;
        z->tile_rows = 4;
    } else if (st == ZDA_OK) {
        zda_status s1 = ZDA_OK;
        for (auto &f : z->F[1]) if (s1 == ZDA_OK) s1 = dev_alloc(z, &f, z->ncell);
        if (s1 == ZDA_OK) s1 = dev_alloc(z, &z->auxR[1], (size_t)N_AUX_R * d->nz * z->dR * d->nphi);
        if (s1 == ZDA_OK) s1 = dev_alloc(z, &z->auxZ[1], (size_t)N_AUX_Z * z->dZ * z->plane);
        if (s1 != ZDA_OK) {
            for (auto &f : z->F[1]) dev_free(z, f);
            dev_free(z, z->auxR[1]);
            dev_free(z, z->auxZ[1]);
            z->fused = false;
            z->tile_rows = 4;
        } else {
            z->has_second = true;
            // intermediate auxiliaries of the two-step kernel (optional)
            zda_status s2 = dev_alloc(z, &z->mauxR, (size_t)N_AUX_R * d->nz * z->dR * d->nphi);
            if (s2 == ZDA_OK) s2 = dev_alloc(z, &z->mauxZ, (size_t)N_AUX_Z * z->dZ * z->plane);
            if (s2 == ZDA_OK && d->nr <= 65535 && d->nz <= 65535) {
                // default two-step shape: 13 owned rows, chunk depth from
                // the launch-round model
                z->has_m = true;
                z->two = true;
                z->fused = false;
                z->tile_rows = 13;
                hipDeviceProp_t prop;
                const int n_cu = hipGetDeviceProperties(&prop, z->device) == hipSuccess && prop.multiProcessorCount > 0
                                     ? prop.multiProcessorCount : 256;
                z->kchunk = default_two_step_kchunk(*d, n_cu);
            } else if (s2 == ZDA_OK) {
                z->has_m = true;   // two-step tiles store rows and planes in 16 bits; not the default here
            } else {
                dev_free(z, z->mauxR);
                dev_free(z, z->mauxZ);
            }
            (void)hipGetLastError();
        }
    }
    // narrow wedges (a few phi cells, down to the continuous zone's one):
    // the tiled kernels would leave most lanes of each wavefront idle, so the
    // in-place kernels with the flat (r, phi) mapping are the default there
    // (measured on 1250-row zones: 11 phi cells 10.2 -> 32.6, 16 cells
    // 14.0 -> 36.2, the continuous zone 1.1 -> 13.2 Gcell-updates/s against
    // the two-step kernel); short chunks, down to 2 planes, while the grid
    // has fewer than 8192 blocks
    if (st == ZDA_OK && narrow) {
        z->fused = false;
        z->two = false;
        z->tile_rows = FLAT_ROWS;
        const long blocks = ((long)d->nr * d->nphi + FLAT_BLOCK_HOST - 1) / FLAT_BLOCK_HOST;
        int kc = std::min(12, d->nz);
        while (kc > 2 && blocks * ((d->nz + kc - 1) / kc) < 8192) --kc;
        z->kchunk = kc;
    } else if (st == ZDA_OK && z->two && d->nphi <= FLAT_TWO_MAX_PHI) {
        // somewhat wider wedges (17 to 32 phi cells): the two-step kernel with
        // the flat mapping in 4-plane chunks (1250 x nphi x 180 zones: 22
        // cells 18.8 -> 30.8, 32 cells 25.6 -> 32.9 Gcell-updates/s against
        // the 13-row two-step kernel; the flat in-place kernels 29.5, 27.7)
        z->tile_rows = FLAT_TWO_ROWS;
        z->kchunk = std::min(4, d->nz);
    }
    if (st == ZDA_OK) st = dev_alloc(z, &z->rows, (size_t)d->nr);
    if (st == ZDA_OK) st = dev_alloc(z, &z->zrows, (size_t)d->nz);
    if (st == ZDA_OK) st = dev_alloc(z, &z->flag, 1);
    if (st == ZDA_OK && hipHostMalloc((void **)&z->flag_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        z->flag_host = nullptr;
        st = fail(ZDA_ERR_OOM, "pinned host allocation failed");
    }
    if (st == ZDA_OK) st = dev_alloc(z, &z->dft_plane, (size_t)ZDA_MAX_FREQ * 2 * z->plane);
    if (st != ZDA_OK) { free_all(z); delete z; return st; }
    if (hipMemcpy(z->rows, rows.data(), rows.size() * sizeof(RowCoef), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(z->zrows, zr.data(), zr.size() * sizeof(ZCoef), hipMemcpyHostToDevice) != hipSuccess) {
        free_all(z); delete z;
        return fail(ZDA_ERR_HIP, "upload of coefficient rows failed");
    }
    // a new zone starts from zero fields, auxiliaries and monitors
    if ((st = reset_state(z, nullptr)) != ZDA_OK) { free_all(z); delete z; return st; }
    launch_fill(z->dft_plane, (size_t)ZDA_MAX_FREQ * 2 * z->plane, nullptr);
    if (hipStreamSynchronize(nullptr) != hipSuccess) { free_all(z); delete z; return fail(ZDA_ERR_HIP, "zone reset failed"); }
    *z->flag_host = 0;
    *out = z;
    if ((st = zda_zone_set_eps(z, eps, eps_on_device)) != ZDA_OK) { zda_zone_destroy(z); *out = nullptr; return st; }
    return ZDA_OK;
}

void zda_zone_destroy(zda_zone *z)
{
    if (!z) return;
    DeviceGuard g(z->device);
    (void)hipDeviceSynchronize();
    free_all(z);
    delete z;
}

zda_status zda_zone_set_eps(zda_zone *z, const float *eps, int on_device)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    DeviceGuard g(z->device);
    hipStream_t s = z->stream;
    // the permittivity lands in the dt/eps array and is converted in place
    if (eps && !on_device)
        HIP_TRY(hipMemcpyAsync(z->ceps, eps, z->ncell * sizeof(float), hipMemcpyHostToDevice, s));
    launch_inv_eps(z->ceps, eps ? (on_device ? eps : z->ceps) : nullptr, z->ncell, z->dt, s);
    HIP_TRY(hipGetLastError());
    if (eps && !on_device) HIP_TRY(hipStreamSynchronize(s));
    return ZDA_OK;
}

zda_status zda_zone_set_design(zda_zone *z, const float *rho, int on_device)
{
    if (!z || !rho) return fail(ZDA_ERR_ARG, "NULL argument");
    if (z->nd <= 0) return fail(ZDA_ERR_STATE, "zone has no design layer");
    DeviceGuard g(z->device);
    hipStream_t s = z->stream;
    const size_t n = (size_t)z->nd * z->plane;
    float *dst = z->ceps + (size_t)z->d.design_k0 * z->plane;
    if (!on_device) HIP_TRY(hipMemcpyAsync(dst, rho, n * sizeof(float), hipMemcpyHostToDevice, s));
    launch_design_dt(dst, on_device ? rho : dst, n, z->d.eps_bg, z->d.eps_hi, z->dt, s);
    HIP_TRY(hipGetLastError());
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    return ZDA_OK;
}

zda_status zda_zone_set_stream(zda_zone *z, void *stream)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    z->stream = (hipStream_t)stream;
    return ZDA_OK;
}

zda_status zda_zone_sync(zda_zone *z)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    DeviceGuard g(z->device);
    HIP_TRY(post_flag(z, z->stream));
    HIP_TRY(zone_wait(z));
    if (*z->flag_host) return fail(ZDA_ERR_DIVERGED, "the watchdog found non-finite or exploding fields");
    return ZDA_OK;
}

zda_status zda_fdtd_run(zda_zone *z, const zda_source *s, int nsteps, const double *omega, int K, int dft_flags,
                        void *stream)
{
    if (!z || !s) return fail(ZDA_ERR_ARG, "NULL zone or source");
    if (z->released) return released_error();
    DeviceGuard g(z->device);
    hipStream_t hs = (hipStream_t)stream;
    z->stream = hs;
    FwdPlan plan;
    RunBufs rb;
    zda_status st = forward_setup(z, s, nsteps, omega, K, dft_flags, hs, plan, rb);
    if (st != ZDA_OK) return st;
    if ((st = run_loop(z, z->d.m, nsteps, s->k_src, plan.P, plan.prof.data(), omega, K, plan.dplane, plan.dvol,
                       plan.reset, hs, rb, (dft_flags & ZDA_RUN_TIMING) != 0)) != ZDA_OK)
        return st;
    forward_finish(z, plan, nsteps, omega, K);
    return ZDA_OK;
}

namespace {

// Device scratch of zda_fdtd_run_noalloc: [pattern | profiles | twiddles |
// tile list], one copy per GPU for the life of the process.  Host code never
// passes `scratch` itself (in host code it is a stand-in, not a device
// address): it uses the address hipGetSymbolAddress returns on each device.
constexpr size_t NA_PATTERN = ZDA_NOALLOC_PATTERN, NA_STEPS = ZDA_NOALLOC_STEPS, NA_TILES = ZDA_NOALLOC_TILES;
constexpr size_t NA_F2 = NA_PATTERN + 2 * NA_STEPS + 2 * NA_TILES;   // float2 units (a tile is two)
static_assert(NA_F2 * sizeof(float2) == ZDA_NOALLOC_SCRATCH_BYTES, "scratch size");

}  // namespace

static __device__ __align__(256) float2 scratch[NA_F2];

namespace {

constexpr int NA_MAX_DEV = 64;
std::mutex g_scratch_mu;
float2 *g_scratch_dev[NA_MAX_DEV] = {};

// the scratch array's address on `dev` (the current device), looked up once
zda_status scratch_on(int dev, float2 **out)
{
    if (dev < 0 || dev >= NA_MAX_DEV) return fail(ZDA_ERR_UNSUPPORTED, "device %d beyond %d", dev, NA_MAX_DEV);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ZDA_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (float2 *)p;
    }
    *out = g_scratch_dev[dev];
    return ZDA_OK;
}

}  // namespace

zda_status zda_fdtd_run_noalloc(zda_zone *z, const zda_source *s, int nsteps, const double *omega, int K,
                                int dft_flags, void *stream)
{
    if (!z || !s) return fail(ZDA_ERR_ARG, "NULL zone or source");
    if (z->released) return released_error();
    if (dft_flags & ZDA_RUN_TIMING) return fail(ZDA_ERR_ARG, "ZDA_RUN_TIMING is not available without allocation");
    if (nsteps < 0 || K < 0 || K > ZDA_MAX_FREQ) return fail(ZDA_ERR_ARG, "bad nsteps or K");
    if (s->k_src < 1 || s->k_src >= z->d.nz) return fail(ZDA_ERR_ARG, "k_src must be in [1, nz)");
    if (s->kind == ZDA_SRC_CUSTOM && (s->n_profiles < 1 || s->n_profiles > ZDA_MAX_FREQ))
        return fail(ZDA_ERR_ARG, "CUSTOM needs 1..%d patterns and profiles", ZDA_MAX_FREQ);
    const size_t P = (size_t)source_patterns(s), T = (size_t)std::max(nsteps, 1);
    if (P * 2 * z->plane > NA_PATTERN)
        return fail(ZDA_ERR_ARG, "%zu pattern samples exceed the no-allocation limit %zu", P * 2 * z->plane,
                    NA_PATTERN);
    if (T * P > NA_STEPS || T * (size_t)std::max(K, 1) > NA_STEPS)
        return fail(ZDA_ERR_ARG, "nsteps %d with %zu profiles and %d frequencies exceeds the no-allocation limit %zu",
                    nsteps, P, K, NA_STEPS);
    DeviceGuard g(z->device);
    float2 *base = nullptr;
    zda_status st = scratch_on(z->device, &base);
    if (st != ZDA_OK) return st;
    RunBufs rb;
    rb.noalloc = true;
    rb.pattern = base;
    rb.cap_pattern = NA_PATTERN;
    rb.profile = base + NA_PATTERN;
    rb.cap_profile = NA_STEPS;
    rb.twiddle = rb.profile + NA_STEPS;
    rb.cap_twiddle = NA_STEPS;
    rb.tiles = (uint4 *)(rb.twiddle + NA_STEPS);
    rb.cap_tiles = NA_TILES;
    TileCounts tc;
    if (z->two) {
        // the tile list depends on the source plane, known before the run
        z->k_src_last = s->k_src;
        plan_zone_tiles(z, z->st_tiles, tc);
        if (z->st_tiles.size() > NA_TILES)
            return fail(ZDA_ERR_ARG, "%zu two-step tiles exceed the no-allocation limit %zu", z->st_tiles.size(),
                        NA_TILES);
    }
    hipStream_t hs = (hipStream_t)stream;
    z->stream = hs;
    FwdPlan plan;
    if ((st = forward_setup(z, s, nsteps, omega, K, dft_flags, hs, plan, rb)) != ZDA_OK) return st;
    if (z->two)
        HIP_TRY(hipMemcpyAsync(rb.tiles, z->st_tiles.data(), z->st_tiles.size() * sizeof(uint4),
                               hipMemcpyHostToDevice, hs));
    if ((st = run_loop(z, z->d.m, nsteps, s->k_src, plan.P, plan.prof.data(), omega, K, plan.dplane, plan.dvol,
                       plan.reset, hs, rb, false, &tc)) != ZDA_OK)
        return st;
    // the next call rewrites the pageable host staging these copies read
    HIP_TRY(hipStreamSynchronize(hs));
    forward_finish(z, plan, nsteps, omega, K);
    return ZDA_OK;
}

namespace {

// The FP64 state of a zone: one in-place set of the six fields, the layer
// auxiliaries, dt/eps, the coefficient rows, the source sheet and the
// exit-plane DFT.
zda_status f64_setup(zda_zone *z, hipStream_t s)
{
    auto &f = z->f64;
    if (f.ready) return ZDA_OK;
    zda_status st;
    for (auto &p : f.F)
        if ((st = dev_alloc(z, &p, z->ncell)) != ZDA_OK) return st;
    if ((st = dev_alloc(z, &f.ceps, z->ncell)) != ZDA_OK) return st;
    if (z->dR > 0 && (st = dev_alloc(z, &f.auxR, (size_t)N_AUX_R * z->d.nz * z->dR * z->d.nphi)) != ZDA_OK)
        return st;
    if (z->dZ > 0 && (st = dev_alloc(z, &f.auxZ, (size_t)N_AUX_Z * z->dZ * z->plane)) != ZDA_OK) return st;
    if ((st = dev_alloc(z, &f.rows, z->rows64.size())) != ZDA_OK) return st;
    if ((st = dev_alloc(z, &f.zrows, z->zrows64.size())) != ZDA_OK) return st;
    if ((st = dev_alloc(z, &f.pattern, 2 * z->plane)) != ZDA_OK) return st;
    if ((st = dev_alloc(z, &f.dft, (size_t)ZDA_MAX_FREQ * 2 * z->plane)) != ZDA_OK) return st;
    HIP_TRY(hipMemcpyAsync(f.rows, z->rows64.data(), z->rows64.size() * sizeof(RowCoefT<double>),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(f.zrows, z->zrows64.data(), z->zrows64.size() * sizeof(ZCoefT<double>),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    f.ready = true;
    return ZDA_OK;
}

}  // namespace

zda_status zda_fdtd_run_fp64(zda_zone *z, const double *eps, int eps_on_device, const zda_source *s, int nsteps,
                             const double *omega, int K, double *plane_out, int out_on_device, void *stream)
{
    if (!z || !eps || !s || !plane_out || (K > 0 && !omega)) return fail(ZDA_ERR_ARG, "NULL argument");
    if (nsteps < 0 || K < 1 || K > ZDA_MAX_FREQ) return fail(ZDA_ERR_ARG, "bad nsteps or K (1..%d)", ZDA_MAX_FREQ);
    const zda_zone_desc &d = z->d;
    if (s->kind != ZDA_SRC_PLANE_CIRC && s->kind != ZDA_SRC_RADIAL)
        return fail(ZDA_ERR_UNSUPPORTED, "FP64 runs take the preset sources only");
    if (s->kind == ZDA_SRC_PLANE_CIRC && std::abs(d.m) != 1) return fail(ZDA_ERR_UNSUPPORTED, "PLANE_CIRC needs |m| = 1");
    if (s->kind == ZDA_SRC_RADIAL && d.m != 0) return fail(ZDA_ERR_UNSUPPORTED, "RADIAL needs m = 0");
    if (!(s->width > 0)) return fail(ZDA_ERR_ARG, "pulse width must be > 0");
    if (s->k_src < 1 || s->k_src >= d.nz) return fail(ZDA_ERR_ARG, "k_src must be in [1, nz)");
    if (d.axis && (d.n_fold > 0 ? d.m % d.n_fold == 0 : d.m == 0))
        return fail(ZDA_ERR_UNSUPPORTED, "axis zone with seam phase 1");
    DeviceGuard g(z->device);
    hipStream_t hs = (hipStream_t)stream;
    z->stream = hs;
    HIP_TRY(zone_wait(z));
    zda_status st = f64_setup(z, hs);
    if (st != ZDA_OK) return st;
    auto &f = z->f64;
    const size_t T = (size_t)std::max(nsteps, 1);
    if (f.cap_steps < T * K || f.cap_steps < T) {
        z->mem.put(f.prof);
        z->mem.put(f.tw);
        f.prof = f.tw = nullptr;
        f.cap_steps = 0;
        if ((st = dev_alloc(z, &f.prof, T * K)) != ZDA_OK) return st;
        if ((st = dev_alloc(z, &f.tw, T * K)) != ZDA_OK) return st;
        f.cap_steps = T * K;
    }
    // dt / eps from the FP64 permittivity
    HIP_TRY(hipMemcpyAsync(f.ceps, eps, z->ncell * sizeof(double),
                           eps_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, hs));
    launch_inv_eps64(f.ceps, f.ceps, z->ncell, z->dt, hs);
    // reset
    for (auto p : f.F) launch_fill64(p, z->ncell, hs);
    if (f.auxR) launch_fill64(f.auxR, (size_t)N_AUX_R * d.nz * z->dR * d.nphi, hs);
    if (f.auxZ) launch_fill64(f.auxZ, (size_t)N_AUX_Z * z->dZ * z->plane, hs);
    launch_fill64(f.dft, (size_t)K * 2 * z->plane, hs);
    // source sheet, pulse and twiddles in FP64 (pageable staging, consumed
    // before the call returns)
    std::vector<double2> pat(2 * z->plane), prof(T), tw(T * K);
    preset_pattern_host(z, s->kind, pat.data());
    const int n0 = s->n0 >= 0 ? s->n0 : default_n0(s->width, z->dt);
    for (size_t n = 0; n < T; ++n) prof[n] = make_double2(n < (size_t)nsteps ? pulse_at((long)n, z->dt, s->omega_c, s->width, n0) : 0.0, 0.0);
    for (size_t n = 0; n < T; ++n)
        for (int k = 0; k < K; ++k) {
            const cd t = z->dt * std::exp(cd(0.0, omega[k] * (double)(n + 1) * z->dt));
            tw[n * K + k] = make_double2(t.real(), t.imag());
        }
    HIP_TRY(hipMemcpyAsync(f.pattern, pat.data(), pat.size() * sizeof(double2), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipMemcpyAsync(f.prof, prof.data(), prof.size() * sizeof(double2), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipMemcpyAsync(f.tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, hs));
    StepArgs64 a{};
    a.nr = d.nr; a.nphi = d.nphi; a.nz = d.nz;
    a.pr0 = d.pml_r_in; a.pr1 = d.pml_r_out; a.pz0 = d.pml_z_lo; a.pz1 = d.pml_z_hi;
    a.dR = z->dR; a.dZ = z->dZ;
    a.dt = z->dt;
    a.inv_dr = 1.0 / d.dr;
    a.inv_dz = 1.0 / d.dz;
    a.cr = z->cr; a.cz = z->cz;
    if (d.n_fold > 0) {
        const double ph = d.m * z->tau;
        a.seam_p = make_double2(std::cos(ph), std::sin(ph));
        a.seam_m = make_double2(std::cos(ph), -std::sin(ph));
    } else {
        a.seam_p = make_double2(1.0, (double)d.m);
        a.seam_m = make_double2(1.0, (double)-d.m);
    }
    a.axis = d.axis ? 1 : 0;
    a.Er = f.F[0]; a.Ep = f.F[1]; a.Ez = f.F[2]; a.Hr = f.F[3]; a.Hp = f.F[4]; a.Hz = f.F[5];
    a.ceps = f.ceps;
    a.auxR = f.auxR; a.auxZ = f.auxZ;
    a.rows = f.rows; a.zrows = f.zrows;
    a.k_src = s->k_src; a.n_prof = 1;
    a.pattern = f.pattern; a.profile = f.prof;
    a.K = K; a.twiddle = f.tw;
    a.k_mon = d.k_mon; a.dft_plane = f.dft;
    a.k0 = d.design_k0; a.k1 = d.design_k1; a.dft_vol = nullptr;
    a.kchunk = std::min(d.nz, 16);
    a.tile_rows = 4;
    for (int n = 0; n < nsteps; ++n) {
        launch_h_step64(a, n, hs);
        launch_e_step64(a, n, hs);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(plane_out, f.dft, (size_t)K * 2 * z->plane * sizeof(double2),
                           out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, hs));
    // the pageable staging above (and a host eps) must be read before it goes
    HIP_TRY(hipStreamSynchronize(hs));
    return ZDA_OK;
}

zda_status zda_dft_fields(zda_zone *z, int monitor, int component_mask, float *out, size_t out_floats,
                          int out_on_device)
{
    if (!z || !out) return fail(ZDA_ERR_ARG, "NULL argument");
    DeviceGuard g(z->device);
    const float2 *src = nullptr;
    size_t block = 0;     // samples of one component at one frequency
    int ncomp = 0;
    if (monitor == ZDA_MON_PLANE) {
        if (!z->have_plane) return fail(ZDA_ERR_STATE, "no plane DFT in the last run");
        src = z->dft_plane;
        block = z->plane;
        ncomp = 2;
    } else if (monitor == ZDA_MON_VOLUME || monitor == ZDA_MON_ADJOINT_VOLUME) {
        const bool adj = monitor == ZDA_MON_ADJOINT_VOLUME;
        if (!(adj ? z->have_vol_adj : z->have_vol)) return fail(ZDA_ERR_STATE, "volume DFT not available");
        src = adj ? z->dft_vol_adj : z->dft_vol;
        block = (size_t)z->nd * z->plane;
        ncomp = 3;
    } else {
        return fail(ZDA_ERR_ARG, "unknown monitor %d", monitor);
    }
    const int all = (1 << ncomp) - 1;
    const int mask = component_mask == 0 ? all : component_mask;
    if (mask & ~all) return fail(ZDA_ERR_ARG, "component mask 0x%x names a component this monitor lacks", component_mask);
    int nsel = 0;
    for (int c = 0; c < ncomp; ++c) nsel += (mask >> c) & 1;
    const int K = z->last_K;
    const size_t n = (size_t)K * nsel * block;
    if (out_floats < 2 * n) return fail(ZDA_ERR_ARG, "output holds %zu floats, %zu needed", out_floats, 2 * n);
    hipStream_t s = z->stream;
    const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    float2 *o = (float2 *)out;
    if (mask == all) {
        HIP_TRY(hipMemcpyAsync(o, src, n * sizeof(float2), kind, s));
    } else {
        for (int k = 0; k < K; ++k)
            for (int c = 0; c < ncomp; ++c)
                if ((mask >> c) & 1) {
                    HIP_TRY(hipMemcpyAsync(o, src + ((size_t)k * ncomp + c) * block, block * sizeof(float2), kind, s));
                    o += block;
                }
    }
    // a monitor that holds non-finite values raises the divergence flag too
    launch_nonfinite(src, (size_t)K * ncomp * block, z->flag, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(post_flag(z, s));
    if (!out_on_device) {
        HIP_TRY(zone_wait(z));
        if (*z->flag_host) return fail(ZDA_ERR_DIVERGED, "non-finite or exploding fields (the run diverged)");
    }
    return ZDA_OK;
}

zda_status zda_adjoint_grad(zda_zone *z, const float *dF_dE, int dF_on_device, float *grad_rho, int grad_on_device,
                            double adj_width, void *stream)
{
    if (!z || !dF_dE || !grad_rho) return fail(ZDA_ERR_ARG, "NULL argument");
    if (z->released) return released_error();
    DeviceGuard g(z->device);
    hipStream_t hs = (hipStream_t)stream;
    z->stream = hs;
    AdjPlan plan;
    zda_status st = adjoint_setup(z, dF_dE, dF_on_device, adj_width, hs, plan);
    if (st != ZDA_OK) return st;
    RunBufs rb;
    rb.pattern = z->pattern;
    if ((st = run_loop(z, -z->d.m, plan.T, z->d.k_mon, plan.K, plan.q.data(), z->last_omega, plan.K, nullptr,
                       z->dft_vol_adj, true, hs, rb)) != ZDA_OK)
        return st;
    return adjoint_finish(z, plan, grad_rho, grad_on_device, hs);
}

zda_status zda_zone_read_field(zda_zone *z, int comp, float *out, int out_on_device)
{
    if (!z || !out || comp < 0 || comp > 5) return fail(ZDA_ERR_ARG, "bad argument");
    if (z->released) return released_error();
    DeviceGuard g(z->device);
    HIP_TRY(hipMemcpyAsync(out, z->F[z->cur][comp], z->ncell * sizeof(float2),
                           out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, z->stream));
    if (!out_on_device) HIP_TRY(zone_wait(z));
    return ZDA_OK;
}

zda_status zda_zone_write_field(zda_zone *z, int comp, const float *in, int in_on_device)
{
    if (!z || !in || comp < 0 || comp > 5) return fail(ZDA_ERR_ARG, "bad argument");
    if (z->released) return released_error();
    DeviceGuard g(z->device);
    hipStream_t s = z->stream;
    HIP_TRY(hipMemcpyAsync(z->F[z->cur][comp], in, z->ncell * sizeof(float2),
                           in_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (comp == 1 && z->dR > 0)
        launch_seed_u(z->auxR[z->cur] + (size_t)AUX_U_EP * z->d.nz * z->dR * z->d.nphi, z->F[z->cur][1], z->d.nr,
                      z->d.nphi, z->d.nz, z->d.pml_r_in, z->d.pml_r_out, (float)z->dt, s);
    HIP_TRY(hipGetLastError());
    if (!in_on_device) HIP_TRY(hipStreamSynchronize(s));
    return ZDA_OK;
}

zda_status zda_zone_release_fields(zda_zone *z)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    if (z->released) return ZDA_OK;
    DeviceGuard g(z->device);
    HIP_TRY(zone_wait(z));   // nothing in flight may still use the memory (nor the caller's buffer)
    free_stepping(z);
    z->released = true;
    z->has_m2 = false;
    z->cur = 0;
    z->n_done = 0;
    return ZDA_OK;
}

zda_status zda_zone_fields_bytes(zda_zone *z, size_t *bytes)
{
    if (!z || !bytes) return fail(ZDA_ERR_ARG, "NULL argument");
    size_t total = 0;
    for_each_stepping(z, [&](float2 *&, size_t n) { total += carved_bytes(n); });
    *bytes = total;
    return ZDA_OK;
}

zda_status zda_zone_acquire_fields(zda_zone *z, void *base, size_t bytes)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    if (!z->released) return ZDA_OK;
    DeviceGuard g(z->device);
    zda_status st = ZDA_OK;
    if (base) {
        size_t need = 0;
        zda_zone_fields_bytes(z, &need);
        if (bytes < need) return fail(ZDA_ERR_ARG, "the buffer holds %zu bytes, the zone needs %zu", bytes, need);
        if ((uintptr_t)base % 256 != 0) return fail(ZDA_ERR_ARG, "the buffer must be 256-byte aligned");
        char *p = (char *)base;
        for_each_stepping(z, [&](float2 *&q, size_t n) {
            q = n ? (float2 *)p : nullptr;
            p += carved_bytes(n);
        });
        z->fields_external = true;
    } else {
        for_each_stepping(z, [&](float2 *&q, size_t n) {
            if (st == ZDA_OK) st = dev_alloc(z, &q, n);
        });
        if (st != ZDA_OK) {
            free_stepping(z);
            return st;
        }
    }
    z->has_m2 = z->three;
    z->released = false;
    // zero fields and auxiliaries, as after a reset
    hipStream_t s = z->stream;
    for_each_stepping(z, [&](float2 *&q, size_t n) {
        if (q) launch_fill(q, n, s);
    });
    HIP_TRY(hipGetLastError());
    return ZDA_OK;
}

zda_status zda_zone_set_launch(zda_zone *z, int kchunk, int tile_rows)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    if (kchunk < 1 || kchunk > z->d.nz) return fail(ZDA_ERR_ARG, "kchunk must be in [1, nz]");
    const bool split = tile_rows == 1 || tile_rows == 2 || tile_rows == 4 || tile_rows == 8 || tile_rows == 16 ||
                       tile_rows == FLAT_ROWS;
    const bool fused = tile_rows == 3 || tile_rows == 7 || tile_rows == 15 || tile_rows == FLAT_FUSED_ROWS;
    const bool three = tile_rows == THREE_STEP_ROWS;
    const bool two = tile_rows == 5 || tile_rows == 13 || tile_rows == FLAT_TWO_ROWS || three;
    if (!split && !fused && !two)
        return fail(ZDA_ERR_ARG, "tile_rows must be 1, 2, 4, 8, 16, 32 (in place), 3, 7, 15, 33 (fused), 5, 13, "
                                 "34 (two-step) or 11 (three-step)");
    if ((fused || two) && !z->has_second) return fail(ZDA_ERR_STATE, "no second buffer set");
    if (two && !z->has_m) return fail(ZDA_ERR_STATE, "no intermediate auxiliaries for the two-step kernel");
    if (two && (z->d.nr > 65535 || z->d.nz > 65535)) return fail(ZDA_ERR_ARG, "two-step tiles need nr, nz <= 65535");
    if (tile_rows == FLAT_FUSED_ROWS && z->d.nphi > FLAT_FUSED_MAX_PHI)
        return fail(ZDA_ERR_ARG, "the flat fused step needs nphi <= %d", FLAT_FUSED_MAX_PHI);
    if (tile_rows == FLAT_TWO_ROWS && z->d.nphi > FLAT_TWO_MAX_PHI)
        return fail(ZDA_ERR_ARG, "the flat two-step kernel needs nphi <= %d", FLAT_TWO_MAX_PHI);
    if (three && !z->has_m2 && z->fields_external)
        return fail(ZDA_ERR_STATE, "the zone steps in a caller's buffer: release it before selecting the three-step "
                                   "kernel");
    if (three && !z->has_m2 && !z->released) {
        // the second intermediate time level of the layer auxiliaries (a
        // released zone gets it with the rest of its memory)
        DeviceGuard g(z->device);
        zda_status st = alloc_m2(z);
        if (st != ZDA_OK) return st;
        z->has_m2 = true;
    }
    z->kchunk = kchunk;
    z->tile_rows = tile_rows;
    z->fused = fused;
    z->two = two;
    z->three = three;
    return ZDA_OK;
}

zda_status zda_zone_set_option(zda_zone *z, int option, int value)
{
    if (!z) return fail(ZDA_ERR_ARG, "NULL zone");
    switch (option) {
    case ZDA_OPT_XCD_REMAP: z->xcd_remap = value ? 1 : 0; return ZDA_OK;
    case ZDA_OPT_NT_STORES: z->nt_stores = value ? 1 : 0; return ZDA_OK;
    case ZDA_OPT_LAYER_STREAM: z->layer_stream = value ? 1 : 0; return ZDA_OK;
    case ZDA_OPT_WATCHDOG:
        if (value < 0) return fail(ZDA_ERR_ARG, "watchdog interval must be >= 0");
        z->watch_every = value;
        return ZDA_OK;
    case ZDA_OPT_LAYER_KCHUNK:
        if (value < -1) return fail(ZDA_ERR_ARG, "layer chunk depth must be >= -1");
        z->layer_kchunk = value;
        return ZDA_OK;
    case ZDA_OPT_LAYER_CARRY:
        if (value < 0 || value > 1) return fail(ZDA_ERR_ARG, "layer carry is 0 or 1");
        z->layer_carry = value;
        return ZDA_OK;
    case ZDA_OPT_TILE_PATCH:
        if (value < 0 || (value != 0 && ((value >> 8) < 1 || (value >> 8) > 255 || (value & 0xff) < 1)))
            return fail(ZDA_ERR_ARG, "tile patch must be 0 or (bands << 8) | columns with both in [1, 255]");
        z->tile_patch = value;
        return ZDA_OK;
    default: return fail(ZDA_ERR_ARG, "unknown option %d", option);
    }
}

zda_status zda_zone_get_info(const zda_zone *z, zda_zone_info *info)
{
    if (!z || !info) return fail(ZDA_ERR_ARG, "NULL argument");
    info->cells = z->ncell;
    info->device_bytes = z->mem.bytes;
    info->dt = z->dt;
    info->cfl = z->cfl;
    info->launch_chunks = (z->d.nz + z->kchunk - 1) / z->kchunk;
    info->kchunk = z->kchunk;
    info->tile_rows = z->tile_rows;
    return ZDA_OK;
}

zda_status zda_plan_two_step_tiles(const zda_zone_desc *d, int tile_rows, int kchunk, int k_src, int order,
                                   uint32_t *out, size_t cap, size_t *ntiles, size_t *n_interior)
{
    if (!d || !ntiles || !n_interior) return fail(ZDA_ERR_ARG, "NULL argument");
    if (d->nr < 1 || d->nphi < 1 || d->nz < 2 || d->nr > 65535 || d->nz > 65535)
        return fail(ZDA_ERR_ARG, "sizes must be in [1, 65535] (nz >= 2)");
    if (d->pml_r_in < 0 || d->pml_r_out < 0 || d->pml_z_lo < 0 || d->pml_z_hi < 0 ||
        2 * std::max(d->pml_r_in, d->pml_r_out) > d->nr || 2 * std::max(d->pml_z_lo, d->pml_z_hi) > d->nz)
        return fail(ZDA_ERR_ARG, "layers must be >= 0 and at most half the extent");
    if (tile_rows != 5 && tile_rows != 13 && tile_rows != FLAT_TWO_ROWS && tile_rows != THREE_STEP_ROWS)
        return fail(ZDA_ERR_ARG, "multi-step tile_rows is 5, 13, 34 or 11 (three-step)");
    if (tile_rows == FLAT_TWO_ROWS && d->nphi > FLAT_TWO_MAX_PHI)
        return fail(ZDA_ERR_ARG, "the flat two-step kernel needs nphi <= %d", FLAT_TWO_MAX_PHI);
    if (kchunk < 1) return fail(ZDA_ERR_ARG, "kchunk must be >= 1");
    const bool carry = order >= 0 && (order & ZDA_PLAN_CARRY) != 0;
    if (order >= 0) order &= ~ZDA_PLAN_CARRY;
    if (order > 1 && ((order >> 8) < 1 || (order >> 8) > 255 || (order & 0xff) < 1))
        return fail(ZDA_ERR_ARG, "tile patch must be (bands << 8) | columns with both in [1, 255]");
    zda_zone z;
    z.d = *d;
    TwoStepTiles t;
    two_step_tiles(&z, two_step_rows(tile_rows, d->nphi), std::min(kchunk, d->nz), k_src, order < 0 ? 0 : order, 0u,
                   t, tile_rows == FLAT_TWO_ROWS, carry, tile_rows == THREE_STEP_ROWS);
    *n_interior = t.v[0].size();
    *ntiles = 0;
    for (int q = 0; q < N_LAY; ++q) *ntiles += t.v[q].size();
    if (!out) return ZDA_OK;
    if (cap < *ntiles) return fail(ZDA_ERR_ARG, "out holds %zu tiles, the plan has %zu", cap, *ntiles);
    size_t p = 0;
    for (int q = 0; q < N_LAY; ++q)
        for (const uint4 &u : t.v[q]) {
            out[4 * p] = u.x;
            out[4 * p + 1] = u.y;
            out[4 * p + 2] = u.z;
            out[4 * p + 3] = (uint32_t)q;
            ++p;
        }
    return ZDA_OK;
}

zda_status zda_zone_last_timing(zda_zone *z, zda_timing *t)
{
    if (!z || !t) return fail(ZDA_ERR_ARG, "NULL argument");
    DeviceGuard g(z->device);
    std::memset(t, 0, sizeof *t);
    if (z->timed_steps == 0) return fail(ZDA_ERR_STATE, "the last run was not timed");
    // the last launch group's events (two streams when the layer tiles ran concurrently)
    HIP_TRY(hipEventSynchronize(z->ev[4 * (size_t)z->timed_steps - 3]));
    HIP_TRY(hipEventSynchronize(z->ev[4 * (size_t)z->timed_steps - 1]));
    for (int n = 0; n < z->timed_steps; ++n) {
        float a = 0.f, b = 0.f;
        if (!z->timed_fused || z->timed_two) HIP_TRY(hipEventElapsedTime(&a, z->ev[4 * n], z->ev[4 * n + 1]));
        HIP_TRY(hipEventElapsedTime(&b, z->ev[4 * n + 2], z->ev[4 * n + 3]));
        if (z->timed_two) {
            t->e_ms += a;        // interior tiles
            t->layer_ms += b;    // tiles with layer cells
        } else {
            t->h_ms += a;
            t->e_ms += b;
        }
    }
    t->h_launches = z->timed_fused ? 0 : z->timed_steps;
    t->steps_per_launch = z->timed_two ? z->timed_depth : 1;
    t->layer_launches = z->timed_two ? z->timed_steps : 0;
    t->e_cells = z->timed_two ? z->timed_tc.cells : z->ncell;
    {
        const size_t mon = (z->d.k_mon >= 0 && z->d.k_mon < z->d.nz) ? z->plane : 0;
        t->e_mon_cells = z->timed_two ? z->timed_tc.mon : mon;
        const size_t src = (z->k_src_last >= 0 && z->k_src_last < z->d.nz) ? z->plane : 0;
        t->e_src_cells = z->timed_two ? z->timed_tc.src : src;
    }
    t->e_launches = z->timed_steps;
    return ZDA_OK;
}

const char *zda_status_str(int status)
{
    switch (status) {
    case ZDA_OK: return "ok";
    case ZDA_ERR_ARG: return "invalid argument";
    case ZDA_ERR_CFL: return "Courant condition violated";
    case ZDA_ERR_UNSUPPORTED: return "unsupported configuration";
    case ZDA_ERR_OOM: return "out of device memory";
    case ZDA_ERR_STATE: return "call out of order";
    case ZDA_ERR_HIP: return "HIP runtime error";
    case ZDA_ERR_DIVERGED: return "simulation diverged";
    default: return "unknown status";
    }
}

const char *zda_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of zones (the lens-scale schedule: many uneven zones stepped in one
// launch per time step, the time loop replayed from a captured HIP graph).

struct zda_batch {
    std::vector<zda_zone *> zones;
    int device = 0;
    bool fused = false;
    int tile_rows = 4;
    StepArgs *tab = nullptr;      // [2][nzones]: both buffer parities
    unsigned *prefix = nullptr;   // [nzones]: first block of each zone
    size_t cap = 0;
    int *n_base = nullptr;        // device step offset advanced inside the graph
    hipStream_t cap_stream = nullptr;
    int graph_steps = 32;         // steps per captured graph (even)
    std::vector<StepArgs> h_tab;
    std::vector<unsigned> h_prefix;
    bool two = false;             // two-step kernel (tile_rows 5, 13 or 34)
    uint4 *tiles = nullptr;       // two-step: interior tiles of every zone, then layer tiles
    size_t cap_tiles = 0;
    DevMem mem;
};

namespace {

bool zone_has_second_set(const zda_zone *z) { return z->has_second; }
bool zone_two_step_ok(const zda_zone *z)
{
    return zone_has_second_set(z) && z->has_m && z->d.nr <= 65535 && z->d.nz <= 65535;
}

// One batched time loop: ab[i][0..1] are zone i's step arguments (prepared).
zda_status batch_loop(zda_batch *b, const std::vector<std::array<StepArgs, 2>> &ab, int nsteps, hipStream_t s)
{
    const int nz = (int)b->zones.size();
    b->h_tab.resize(2 * (size_t)nz);
    b->h_prefix.resize(nz);
    unsigned total = 0;
    for (int i = 0; i < nz; ++i) {
        b->h_tab[i] = ab[i][0];
        b->h_tab[nz + i] = ab[i][1];
        b->h_prefix[i] = total;
        if (!b->two) total += b->fused ? tiles_fused(ab[i][0], b->tile_rows) : tiles_split(ab[i][0], b->tile_rows);
    }
    unsigned n_lay[N_LAY] = {};
    if (b->two) {
        // layer tiles with carried auxiliaries as the first zone's option says
        const bool flat = b->tile_rows == FLAT_TWO_ROWS;
        const bool carry = !flat && b->zones[0]->layer_carry != 0;
        TwoStepTiles t;
        for (int i = 0; i < nz; ++i) {
            const zda_zone *z = b->zones[i];
            two_step_tiles(z, two_step_rows(b->tile_rows, z->d.nphi), z->kchunk, ab[i][0].k_src, tile_order(z),
                           (unsigned)i, t, flat, carry);
        }
        std::vector<uint4> all;
        for (int q = 0; q < N_LAY; ++q) {
            n_lay[q] = (unsigned)t.v[q].size();
            all.insert(all.end(), t.v[q].begin(), t.v[q].end());
        }
        if (all.size() > b->cap_tiles) {
            HIP_TRY(hipStreamSynchronize(s));
            b->mem.put(b->tiles);
            b->cap_tiles = 0;
            b->tiles = (uint4 *)b->mem.get(all.size() * sizeof(uint4));
            if (!b->tiles) return fail(ZDA_ERR_OOM, "device allocation of the batch tile list failed");
            b->cap_tiles = all.size();
        }
        HIP_TRY(hipMemcpyAsync(b->tiles, all.data(), all.size() * sizeof(uint4), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));   // the staging vector goes out of scope
    }
    if ((size_t)nz > b->cap) {
        HIP_TRY(hipStreamSynchronize(s));
        b->mem.put(b->tab);
        b->mem.put(b->prefix);
        b->cap = 0;
        b->tab = (StepArgs *)b->mem.get(2 * (size_t)nz * sizeof(StepArgs));
        b->prefix = (unsigned *)b->mem.get((size_t)nz * sizeof(unsigned));
        if (!b->tab || !b->prefix) return fail(ZDA_ERR_OOM, "device allocation of the batch tables failed");
        b->cap = nz;
    }
    HIP_TRY(hipMemcpyAsync(b->tab, b->h_tab.data(), b->h_tab.size() * sizeof(StepArgs), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->prefix, b->h_prefix.data(), nz * sizeof(unsigned), hipMemcpyHostToDevice, s));
    launch_set_int(b->n_base, 0, s);
    HIP_TRY(hipStreamSynchronize(s));
    BatchArgs ba[2];
    for (int p = 0; p < 2; ++p) {
        ba[p].tab = b->tab + (size_t)p * nz;
        ba[p].prefix = b->prefix;
        ba[p].nzones = nz;
        ba[p].n_base = b->n_base;
        ba[p].xcd_remap = b->zones[0]->xcd_remap;
        ba[p].tiles = b->tiles;
    }
    // steps q and q+1 of the two-step kernel: interior tiles of every zone,
    // then their layer tiles; the pair alternates buffer parities
    auto two_pair = [&](int q, hipStream_t st) {
        BatchArgs x = ba[(q / 2) & 1];
        size_t off = 0;
        for (int l = 0; l < N_LAY; ++l) {
            x.tiles = b->tiles + off;
            launch_batch_two(x, n_lay[l], b->tile_rows, l, q, st);
            off += n_lay[l];
        }
    };
    const int S = b->graph_steps;
    const int reps = nsteps >= 2 * S ? nsteps / S : 0;
    if (reps > 0) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        // the fused step alternates buffer parities; the split kernels update one set in place
        if (b->two) {
            for (int q = 0; q < S; q += 2) two_pair(q, b->cap_stream);
        } else {
            for (int q = 0; q < S; ++q)
                launch_batch_step(ba[b->fused ? (q & 1) : 0], total, b->tile_rows, b->fused, q, b->cap_stream);
        }
        launch_advance_step(b->n_base, S, b->cap_stream);
        HIP_TRY(hipStreamEndCapture(b->cap_stream, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(ZDA_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        // after whole graphs every zone is back on the buffer set its run
        // started from (each graph holds an even number of steps); the
        // watchdog checks those fields every watch_every steps
        const long W = b->zones[0]->watch_every;
        long next_watch = W > 0 ? ((long)b->zones[0]->n_done / W + 1) * W : -1;
        for (int q = 0; q < reps && e == hipSuccess; ++q) {
            e = hipGraphLaunch(exec, s);
            const long at = (long)b->zones[0]->n_done + (long)(q + 1) * S;
            if (e == hipSuccess && W > 0 && at >= next_watch) {
                for (int i = 0; i < nz; ++i) {
                    WatchArgs w{};
                    const StepArgs &a0 = ab[i][0];
                    w.f[0] = a0.Er; w.f[1] = a0.Ep; w.f[2] = a0.Ez;
                    w.f[3] = a0.Hr; w.f[4] = a0.Hp; w.f[5] = a0.Hz;
                    w.n = b->zones[i]->ncell;
                    w.flag = b->zones[i]->flag;
                    w.bound2 = WATCH_BOUND2;
                    launch_watch(w, s);
                }
                while (next_watch <= at) next_watch += W;
                e = hipGetLastError();
            }
        }
        hipError_t e2 = hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(ZDA_ERR_HIP, "graph launch: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const int done = reps * S;
    if (b->two) {
        int q = 0;
        for (; q + 1 < nsteps - done; q += 2) two_pair(q, s);
        if (q < nsteps - done) {
            // an odd last step: the fused step of each zone (absolute step index)
            for (int i = 0; i < nz; ++i) {
                StepArgs a1 = ab[i][((nsteps - done) / 2) & 1];
                a1.tile_rows = b->tile_rows == FLAT_TWO_ROWS ? FLAT_FUSED_ROWS : 3;
                launch_fused_step(a1, nsteps - 1, s);
            }
        }
    } else {
        for (int q = 0; q < nsteps - done; ++q)
            launch_batch_step(ba[b->fused ? (q & 1) : 0], total, b->tile_rows, b->fused, q, s);
    }
    HIP_TRY(hipGetLastError());
    const int flips = b->two ? nsteps / 2 + (nsteps & 1) : (b->fused ? nsteps : 0);
    for (auto z : b->zones) {
        z->n_done += nsteps;
        z->cur ^= (flips & 1);
        HIP_TRY(post_flag(z, s));
    }
    return ZDA_OK;
}

}  // namespace

extern "C" {

zda_status zda_batch_create(zda_zone *const *zones, int nzones, zda_batch **out)
{
    if (!zones || nzones < 1 || !out) return fail(ZDA_ERR_ARG, "need at least one zone and an output pointer");
    *out = nullptr;
    for (int i = 0; i < nzones; ++i)
        if (!zones[i]) return fail(ZDA_ERR_ARG, "zone %d is NULL", i);
    const int dev = zones[0]->device;
    for (int i = 1; i < nzones; ++i)
        if (zones[i]->device != dev) return fail(ZDA_ERR_ARG, "zones must live on one device");
    zda_batch *b = new (std::nothrow) zda_batch();
    if (!b) return fail(ZDA_ERR_OOM, "host allocation failed");
    b->zones.assign(zones, zones + nzones);
    b->device = dev;
    b->fused = true;
    for (auto z : b->zones) b->fused = b->fused && zone_has_second_set(z);
    b->tile_rows = b->fused ? 3 : 4;
    DeviceGuard g(dev);
    b->mem.al = current_allocator();
    b->mem.device = dev;
    b->n_base = (int *)b->mem.get(sizeof(int));
    if (!b->n_base || hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        zda_batch_destroy(b);
        return fail(ZDA_ERR_HIP, "batch setup failed");
    }
    *out = b;
    return ZDA_OK;
}

void zda_batch_destroy(zda_batch *b)
{
    if (!b) return;
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
    b->mem.put_all();
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

zda_status zda_batch_set_launch(zda_batch *b, int tile_rows, const int *kchunk)
{
    if (!b) return fail(ZDA_ERR_ARG, "NULL batch");
    const bool split = tile_rows == 1 || tile_rows == 2 || tile_rows == 4 || tile_rows == 8 || tile_rows == 16 ||
                       tile_rows == FLAT_ROWS;
    const bool fused = tile_rows == 3 || tile_rows == 7 || tile_rows == 15 || tile_rows == FLAT_FUSED_ROWS;
    const bool two = tile_rows == 5 || tile_rows == 13 || tile_rows == FLAT_TWO_ROWS;
    if (!split && !fused && !two)
        return fail(ZDA_ERR_ARG, "tile_rows must be 1, 2, 4, 8, 16, 32 (in place), 3, 7, 15, 33 (fused) or 5, 13, "
                                 "34 (two-step)");
    if (tile_rows == FLAT_TWO_ROWS)
        for (auto z : b->zones)
            if (z->d.nphi > FLAT_TWO_MAX_PHI)
                return fail(ZDA_ERR_ARG, "the flat two-step kernel needs nphi <= %d", FLAT_TWO_MAX_PHI);
    if (fused)
        for (auto z : b->zones)
            if (!zone_has_second_set(z)) return fail(ZDA_ERR_STATE, "a zone has no second buffer set");
    if (tile_rows == FLAT_FUSED_ROWS)
        for (auto z : b->zones)
            if (z->d.nphi > FLAT_FUSED_MAX_PHI)
                return fail(ZDA_ERR_ARG, "the flat fused step needs nphi <= %d", FLAT_FUSED_MAX_PHI);
    if (two)
        for (auto z : b->zones)
            if (!zone_two_step_ok(z)) return fail(ZDA_ERR_STATE, "a zone cannot run the two-step kernel");
    if (kchunk)
        for (size_t i = 0; i < b->zones.size(); ++i)
            if (kchunk[i] < 1 || kchunk[i] > b->zones[i]->d.nz) return fail(ZDA_ERR_ARG, "kchunk[%zu] out of range", i);
    b->fused = fused;
    b->two = two;
    b->tile_rows = tile_rows;
    if (kchunk)
        for (size_t i = 0; i < b->zones.size(); ++i) b->zones[i]->kchunk = kchunk[i];
    return ZDA_OK;
}

zda_status zda_batch_run(zda_batch *b, const zda_source *sources, int nsteps, const double *omega, int K,
                         int dft_flags, void *stream)
{
    if (!b || !sources) return fail(ZDA_ERR_ARG, "NULL batch or sources");
    if (dft_flags & ZDA_RUN_TIMING) return fail(ZDA_ERR_ARG, "per-kernel timing is not available for batches");
    for (auto z : b->zones)
        if (z->released) return released_error();
    DeviceGuard g(b->device);
    hipStream_t hs = (hipStream_t)stream;
    const size_t nz = b->zones.size();
    std::vector<FwdPlan> plans(nz);
    std::vector<RunBufs> rbs(nz);
    std::vector<std::array<StepArgs, 2>> ab(nz);
    zda_status st;
    for (size_t i = 0; i < nz; ++i) {
        zda_zone *z = b->zones[i];
        z->stream = hs;
        if ((st = forward_setup(z, &sources[i], nsteps, omega, K, dft_flags, hs, plans[i], rbs[i])) != ZDA_OK)
            return st;
        if ((st = prepare_run(z, z->d.m, nsteps, sources[i].k_src, plans[i].P, plans[i].prof.data(), omega, K,
                              plans[i].dplane, plans[i].dvol, plans[i].reset, hs, ab[i].data(), rbs[i])) != ZDA_OK)
            return st;
    }
    if ((st = batch_loop(b, ab, nsteps, hs)) != ZDA_OK) return st;
    for (size_t i = 0; i < nz; ++i) forward_finish(b->zones[i], plans[i], nsteps, omega, K);
    return ZDA_OK;
}

zda_status zda_batch_adjoint_grad(zda_batch *b, const float *const *dF_dE, float *const *grad_rho, void *stream)
{
    if (!b || !dF_dE || !grad_rho) return fail(ZDA_ERR_ARG, "NULL argument");
    DeviceGuard g(b->device);
    hipStream_t hs = (hipStream_t)stream;
    const size_t nz = b->zones.size();
    int T = -1;
    for (auto z : b->zones) {
        if (z->released) return released_error();
        if (!z->have_vol || z->last_K < 1) return fail(ZDA_ERR_STATE, "every zone needs a forward run with ZDA_DFT_VOLUME");
        if (T >= 0 && z->last_T != T) return fail(ZDA_ERR_STATE, "zones ran different step counts");
        T = z->last_T;
    }
    std::vector<AdjPlan> plans(nz);
    std::vector<std::array<StepArgs, 2>> ab(nz);
    zda_status st;
    for (size_t i = 0; i < nz; ++i) {
        zda_zone *z = b->zones[i];
        if (!dF_dE[i] || !grad_rho[i]) return fail(ZDA_ERR_ARG, "NULL pointer for zone %zu", i);
        z->stream = hs;
        if ((st = adjoint_setup(z, dF_dE[i], 1, 0.0, hs, plans[i])) != ZDA_OK) return st;
        RunBufs rb;
        rb.pattern = z->pattern;
        if ((st = prepare_run(z, -z->d.m, plans[i].T, z->d.k_mon, plans[i].K, plans[i].q.data(), z->last_omega,
                              plans[i].K, nullptr, z->dft_vol_adj, true, hs, ab[i].data(), rb)) != ZDA_OK)
            return st;
    }
    if ((st = batch_loop(b, ab, T, hs)) != ZDA_OK) return st;
    for (size_t i = 0; i < nz; ++i)
        if ((st = adjoint_finish(b->zones[i], plans[i], grad_rho[i], 1, hs)) != ZDA_OK) return st;
    return ZDA_OK;
}

zda_status zda_batch_autotune(zda_batch *b, const zda_source *sources, int probe_steps, const double *omega, int K,
                              void *stream, zda_tune_result *res)
{
    if (!b || !sources || !res || probe_steps < 2) return fail(ZDA_ERR_ARG, "bad autotune arguments");
    for (auto z : b->zones)
        if (z->released) return released_error();
    DeviceGuard g(b->device);
    hipStream_t hs = (hipStream_t)stream;
    const size_t nz = b->zones.size();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EventPair {
        hipEvent_t &a, &b;
        ~EventPair()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int probes = 0;
    auto probe = [&](double &ms) -> zda_status {
        HIP_TRY(hipEventRecord(e0, hs));
        zda_status st = zda_batch_run(b, sources, probe_steps, omega, K, ZDA_DFT_PLANE, stream);
        if (st != ZDA_OK) return st;
        HIP_TRY(hipEventRecord(e1, hs));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        ms = t / probe_steps;
        ++probes;
        return ZDA_OK;
    };
    // 1) kernel family and tile shape with each zone's default depth
    // (the time-block depth: 1 for the split and fused kernels, 2 for the
    // two-step kernel)
    std::vector<int> rows_c = {2, 4, 8, FLAT_ROWS};
    bool can_fuse = true, can_two = true, narrow = true;
    for (auto z : b->zones) {
        can_fuse = can_fuse && zone_has_second_set(z);
        can_two = can_two && zone_two_step_ok(z);
        narrow = narrow && z->d.nphi <= FLAT_TWO_MAX_PHI;
    }
    if (can_fuse) rows_c.insert(rows_c.end(), {3, 7, 15});
    if (can_two) rows_c.insert(rows_c.end(), {5, 13});
    if (can_two && narrow) rows_c.push_back(FLAT_TWO_ROWS);
    // the flat two-step kernel is probed with 16-plane chunks (the zones'
    // own depth suits their default in-place kernels, 2 planes for narrow
    // zones, and would hide it behind its chunk halo)
    std::vector<int> kc(nz), kc_flat(nz);
    for (size_t i = 0; i < nz; ++i) {
        kc[i] = b->zones[i]->kchunk;
        kc_flat[i] = std::min(16, b->zones[i]->d.nz);
    }
    auto depths_of = [&](int rr) { return rr == FLAT_TWO_ROWS ? kc_flat.data() : kc.data(); };
    double best = 1e300;
    int best_rows = b->tile_rows;
    zda_status st;
    for (int rr : rows_c) {
        if ((st = zda_batch_set_launch(b, rr, depths_of(rr))) != ZDA_OK) return st;
        double ms;
        if ((st = probe(ms)) != ZDA_OK) return st;
        if (ms < best) { best = ms; best_rows = rr; }
    }
    if (best_rows == FLAT_TWO_ROWS) kc = kc_flat;
    if ((st = zda_batch_set_launch(b, best_rows, kc.data())) != ZDA_OK) return st;
    // 2) z-chunk depth per size class (thirds of the zones by cell count)
    std::vector<size_t> order(nz);
    for (size_t i = 0; i < nz; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t c) { return b->zones[a]->ncell < b->zones[c]->ncell; });
    const int nclass = nz >= 3 ? 3 : (int)nz;
    for (int cl = 0; cl < nclass; ++cl) {
        const size_t lo = nz * cl / nclass, hi = nz * (cl + 1) / nclass;
        const std::vector<int> kc0 = kc;
        int best_depth = 0;
        const bool two_rows = best_rows == 5 || best_rows == 13 || best_rows == FLAT_TWO_ROWS;
        // the flat two-step kernel measured best at 4-plane chunks on one
        // narrow zone and at 16-24 on a 16-zone lens
        const std::vector<int> depths = best_rows == FLAT_TWO_ROWS ? std::vector<int>{4, 8, 16, 24, 48}
                                        : two_rows                 ? std::vector<int>{16, 24, 32, 48, 96}
                                                                   : std::vector<int>{6, 8, 12, 20, 40};
        for (int depth : depths) {
            for (size_t q = lo; q < hi; ++q) kc[order[q]] = std::min(depth, b->zones[order[q]]->d.nz);
            if ((st = zda_batch_set_launch(b, best_rows, kc.data())) != ZDA_OK) return st;
            double ms;
            if ((st = probe(ms)) != ZDA_OK) return st;
            if (ms < best) { best = ms; best_depth = depth; }
        }
        kc = kc0;
        if (best_depth > 0)
            for (size_t q = lo; q < hi; ++q) kc[order[q]] = std::min(best_depth, b->zones[order[q]]->d.nz);
        if ((st = zda_batch_set_launch(b, best_rows, kc.data())) != ZDA_OK) return st;
    }
    res->tile_rows = best_rows;
    res->ms_per_step = best;
    res->probes = probes;
    return ZDA_OK;
}

}  // extern "C"
