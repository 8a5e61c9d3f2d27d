// zda_kernels.hip -- gfx950 kernels of the ZDA zone library.
//
// The H and E half-steps of the cylindrical Yee leap-frog (eq. 3-5 of arXiv
// 2501.07979, section on the cylindrical solver) for one n-fold Bloch wedge.
// Each thread owns one (i, j) column and marches through a chunk of z-planes,
// keeping the column's previous/next plane in registers; phi is the fastest
// index so a 64-lane wavefront reads 64 consecutive complex samples (512 B)
// per access.  The E half-step fuses the soft source sheet and the exit-plane
// and design-volume DFT accumulation, so the fields are read once per step.
//
// PML: complex stretch of radial lengths (1 + sigma F), radii (1 + Sigma/r F)
// and axial lengths; each stretched term x is divided by its stretch with one
// auxiliary recursion y = g1 x - g2 u, u <- c u + dt y (F is the causal
// one-pole filter dt / (1 - c e^{i w dt})).
#include <type_traits>

#include "zda_internal.h"

namespace zda {

namespace {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_fma(float2 acc, float2 a, float2 b)   // acc + a*b
{
    return make_float2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 zero2() { return make_float2(0.f, 0.f); }

// the same complex helpers in FP64 (the in-place kernels' verification instantiation)
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_fma(double2 acc, double2 a, double2 b)
{
    return make_double2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 mk(double x, double y) { return make_double2(x, y); }
template <typename C>
__device__ __forceinline__ C czero()
{
    C c;
    c.x = 0;
    c.y = 0;
    return c;
}

// y = x / (1 + s F) with the auxiliary u = F y
template <typename C, typename R>
__device__ __forceinline__ C div_stretch(C x, C *aux, R g1, R g2, R c, R dt)
{
    C u = *aux;
    C y = mk(g1 * x.x - g2 * u.x, g1 * x.y - g2 * u.y);
    *aux = mk(c * u.x + dt * y.x, c * u.y + dt * y.y);
    return y;
}

__device__ __forceinline__ int slab_row(int q, int n, int d0, int d1)
{
    if (q < d0) return q;
    if (q >= n - d1) return d0 + (q - (n - d1));
    return -1;
}

constexpr int BX = 64;   // one wavefront along phi
// flat mapping of the in-place kernels: a block of FLAT_BLOCK threads covers
// consecutive cells of the (r, phi) plane (row-major, so still one contiguous
// segment per wavefront); narrow wedges (few phi cells) keep every lane busy
constexpr int FLAT_BLOCK = FLAT_BLOCK_HOST;

// (i, j) of this thread in the in-place kernels, false if outside the zone
template <int BY, bool FLAT, typename A>
__device__ __forceinline__ bool split_cell(const A &a, int bx, int by, int &i, int &j)
{
    if constexpr (FLAT) {
        const unsigned q = (unsigned)bx * FLAT_BLOCK + threadIdx.x;
        if (q >= (unsigned)a.nr * (unsigned)a.nphi) return false;
        i = (int)(q / (unsigned)a.nphi);
        j = (int)(q - (unsigned)i * (unsigned)a.nphi);
        return true;
    } else {
        j = bx * BX + threadIdx.x;
        i = by * BY + threadIdx.y;
        return j < a.nphi && i < a.nr;
    }
}

// H^{n+1/2} = H^{n-1/2} - dt curlE(E^n); also advances V = F H_phi in the r-layer.
template <int BY, bool FLAT = false, typename R = float>
__device__ __forceinline__ void h_step_body(const StepArgsT<R> &a, int n, int bx, int by, int bz)
{
    using C = typename CplxOf<R>::T;
    int i, j;
    if (!split_cell<BY, FLAT>(a, bx, by, i, j)) return;
    const int kb = bz * a.kchunk;
    const int ke = min(kb + a.kchunk, a.nz);
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    const int ir = slab_row(i, nr, a.pr0, a.pr1);
    const int ir1 = (i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoefT<R> rc = a.rows[i];
    const int jp = (j + 1 < nphi) ? j + 1 : 0;
    const bool wrap = (j + 1 >= nphi);
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const R dt = a.dt;

    size_t c = ((size_t)kb * nr + i) * nphi + j;
    C er = a.Er[c], ep = a.Ep[c];
    for (int k = kb; k < ke; ++k, c += plane) {
        const size_t row = c - j;
        const C ez = a.Ez[c];
        C er_kp = czero<C>(), ep_kp = czero<C>();
        if (k + 1 < nz) { er_kp = a.Er[c + plane]; ep_kp = a.Ep[c + plane]; }
        C ez_jp = a.Ez[row + jp], er_jp = a.Er[row + jp];
        if (wrap) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
        C ez_ip = czero<C>(), ep_ip = czero<C>();
        if (i + 1 < nr) { ez_ip = a.Ez[c + nphi]; ep_ip = a.Ep[c + nphi]; }
        const int kz = slab_row(k, nz, a.pz0, a.pz1);
        const size_t sr = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi + j : 0;
        const size_t sz = kz >= 0 ? ((size_t)kz * nr + i) * nphi + j : 0;
        const ZCoefT<R> zc = a.zrows[k];

        // H_r at (i, j+1/2, k+1/2); row 0 is a wall unless it borders the axis
        if (i > 0 || a.axis) {
            C t1 = c_scale(c_sub(ez_jp, ez), rc.inv_rdphi_int);
            C t2 = c_scale(c_sub(ep_kp, ep), a.inv_dz);
            if (ir >= 0) t1 = div_stretch(t1, a.auxR + AUX_HR_T * slabR + sr, rc.g1_t_int, rc.g2_t_int, a.cr, dt);
            if (kz >= 0) t2 = div_stretch(t2, a.auxZ + ZAUX_HR * slabZ + sz, zc.g1_half, zc.g2_half, a.cz, dt);
            C h = a.Hr[c];
            a.Hr[c] = mk(h.x - dt * (t1.x - t2.x), h.y - dt * (t1.y - t2.y));
        }
        // H_phi at (i+1/2, j, k+1/2)
        {
            C t1 = c_scale(c_sub(er_kp, er), a.inv_dz);
            C t2 = c_scale(c_sub(ez_ip, ez), a.inv_dr);
            if (kz >= 0) t1 = div_stretch(t1, a.auxZ + ZAUX_HP * slabZ + sz, zc.g1_half, zc.g2_half, a.cz, dt);
            if (ir >= 0) t2 = div_stretch(t2, a.auxR + AUX_HP_S * slabR + sr, rc.g1_s_half, rc.g2_s_half, a.cr, dt);
            C h = a.Hp[c];
            h = mk(h.x - dt * (t1.x - t2.x), h.y - dt * (t1.y - t2.y));
            a.Hp[c] = h;
            if (ir >= 0) {
                C *v = a.auxR + AUX_V_HP * slabR + sr;
                C vv = *v;
                *v = mk(a.cr * vv.x + dt * h.x, a.cr * vv.y + dt * h.y);
            }
        }
        // H_z at (i+1/2, j+1/2, k)
        if (k > 0) {
            C t = c_add(c_scale(c_sub(ep_ip, ep), a.inv_dr), c_scale(c_add(ep_ip, ep), rc.inv_2r_half));
            if (ir >= 0) {
                const C *U = a.auxR + AUX_U_EP * slabR;
                C u0 = U[sr];
                C u1 = ir1 >= 0 ? U[((size_t)k * a.dR + ir1) * nphi + j] : czero<C>();
                t = c_add(t, c_sub(c_scale(u1, rc.hz_c1), c_scale(u0, rc.hz_c0)));
                t = div_stretch(t, a.auxR + AUX_HZ_S * slabR + sr, rc.g1_s_half, rc.g2_s_half, a.cr, dt);
            }
            t = c_sub(t, c_scale(c_sub(er_jp, er), rc.inv_rdphi_half));
            if (ir >= 0) t = div_stretch(t, a.auxR + AUX_HZ_T * slabR + sr, rc.g1_t_half, rc.g2_t_half, a.cr, dt);
            C h = a.Hz[c];
            a.Hz[c] = mk(h.x - dt * t.x, h.y - dt * t.y);
        }
        er = er_kp;
        ep = ep_kp;
    }
}

// E^{n+1} = E^n + (dt/eps)(curlH(H^{n+1/2}) - J^{n+1/2}); source sheet, DFT
// accumulation and U = F E_phi in the r-layer fused.
template <int BY, bool FLAT = false, typename R = float>
__device__ __forceinline__ void e_step_body(const StepArgsT<R> &a, int n, int bx, int by, int bz)
{
    using C = typename CplxOf<R>::T;
    int i, j;
    if (!split_cell<BY, FLAT>(a, bx, by, i, j)) return;
    const int kb = bz * a.kchunk;
    const int ke = min(kb + a.kchunk, a.nz);
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    const int ir = slab_row(i, nr, a.pr0, a.pr1);
    const int irm = (i > 0) ? slab_row(i - 1, nr, a.pr0, a.pr1) : -1;
    const RowCoefT<R> rc = a.rows[i];
    const int jm = (j > 0) ? j - 1 : nphi - 1;
    const bool wrap = (j == 0);
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const R dt = a.dt;
    const int nd = a.k1 - a.k0;

    size_t c = ((size_t)kb * nr + i) * nphi + j;
    C hp_km = czero<C>(), hr_km = czero<C>();
    if (kb > 0) { hp_km = a.Hp[c - plane]; hr_km = a.Hr[c - plane]; }
    for (int k = kb; k < ke; ++k, c += plane) {
        const size_t row = c - j;
        const C hr = a.Hr[c], hp = a.Hp[c], hz = a.Hz[c];
        C hz_jm = a.Hz[row + jm], hr_jm = a.Hr[row + jm];
        if (wrap) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
        C hz_im = czero<C>(), hp_im = czero<C>();
        if (i > 0) { hz_im = a.Hz[c - nphi]; hp_im = a.Hp[c - nphi]; }
        const R ce = a.ceps[c];
        const int kz = slab_row(k, nz, a.pz0, a.pz1);
        const size_t sr = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi + j : 0;
        const size_t sz = kz >= 0 ? ((size_t)kz * nr + i) * nphi + j : 0;
        const ZCoefT<R> zc = a.zrows[k];
        C jr = czero<C>(), jp = czero<C>();
        if (k == a.k_src) {
            for (int p = 0; p < a.n_prof; ++p) {
                const C g = a.profile[(size_t)n * a.n_prof + p];
                const C *pat = a.pattern + (size_t)p * 2 * plane + (size_t)i * nphi + j;
                jr = c_fma(jr, pat[0], g);
                jp = c_fma(jp, pat[plane], g);
            }
        }
        C er = a.Er[c], ep = a.Ep[c], ez = a.Ez[c];
        // E_r at (i+1/2, j, k)
        if (k > 0) {
            C t1 = c_scale(c_sub(hz, hz_jm), rc.inv_rdphi_half);
            C t2 = c_scale(c_sub(hp, hp_km), a.inv_dz);
            if (ir >= 0) t1 = div_stretch(t1, a.auxR + AUX_ER_T * slabR + sr, rc.g1_t_half, rc.g2_t_half, a.cr, dt);
            if (kz >= 0) t2 = div_stretch(t2, a.auxZ + ZAUX_ER * slabZ + sz, zc.g1_int, zc.g2_int, a.cz, dt);
            er = mk(er.x + ce * (t1.x - t2.x - jr.x), er.y + ce * (t1.y - t2.y - jr.y));
            a.Er[c] = er;
        }
        // E_phi at (i, j+1/2, k) (H_z on the axis is zero)
        if (k > 0 && (i > 0 || a.axis)) {
            C t1 = c_scale(c_sub(hr, hr_km), a.inv_dz);
            C t2 = c_scale(c_sub(hz, hz_im), a.inv_dr);
            if (kz >= 0) t1 = div_stretch(t1, a.auxZ + ZAUX_EP * slabZ + sz, zc.g1_int, zc.g2_int, a.cz, dt);
            if (ir >= 0) t2 = div_stretch(t2, a.auxR + AUX_EP_S * slabR + sr, rc.g1_s_int, rc.g2_s_int, a.cr, dt);
            ep = mk(ep.x + ce * (t1.x - t2.x - jp.x), ep.y + ce * (t1.y - t2.y - jp.y));
            a.Ep[c] = ep;
        }
        // U = F E_phi advances on every r-layer cell (also where E_phi is held)
        if (ir >= 0) {
            C *u = a.auxR + AUX_U_EP * slabR + sr;
            C uu = *u;
            *u = mk(a.cr * uu.x + dt * ep.x, a.cr * uu.y + dt * ep.y);
        }
        // E_z at (i, j, k+1/2) (next to the axis the H_phi term at r = 0 has weight 0)
        if (i > 0 || a.axis) {
            C t = c_add(c_scale(c_sub(hp, hp_im), a.inv_dr), c_scale(c_add(hp, hp_im), rc.inv_2r_int));
            if (ir >= 0) {
                const C *V = a.auxR + AUX_V_HP * slabR;
                C v1 = V[sr];
                C v0 = irm >= 0 ? V[((size_t)k * a.dR + irm) * nphi + j] : czero<C>();
                t = c_add(t, c_sub(c_scale(v1, rc.ez_c1), c_scale(v0, rc.ez_c0)));
                t = div_stretch(t, a.auxR + AUX_EZ_S * slabR + sr, rc.g1_s_int, rc.g2_s_int, a.cr, dt);
            }
            t = c_sub(t, c_scale(c_sub(hr, hr_jm), rc.inv_rdphi_int));
            if (ir >= 0) t = div_stretch(t, a.auxR + AUX_EZ_T * slabR + sr, rc.g1_t_int, rc.g2_t_int, a.cr, dt);
            ez = mk(ez.x + ce * t.x, ez.y + ce * t.y);
            a.Ez[c] = ez;
        }
        // DFT monitors: Ehat += dt e^{i w (n+1) dt} E^{n+1}
        if (a.dft_plane && k == a.k_mon) {
            for (int f = 0; f < a.K; ++f) {
                const C tw = a.twiddle[(size_t)n * a.K + f];
                C *o = a.dft_plane + (size_t)f * 2 * plane + (size_t)i * nphi + j;
                o[0] = c_fma(o[0], tw, er);
                o[plane] = c_fma(o[plane], tw, ep);
            }
        }
        if (a.dft_vol && k >= a.k0 && k < a.k1) {
            const size_t vs = (size_t)nd * plane;
            for (int f = 0; f < a.K; ++f) {
                const C tw = a.twiddle[(size_t)n * a.K + f];
                C *o = a.dft_vol + (size_t)f * 3 * vs + (size_t)(k - a.k0) * plane + (size_t)i * nphi + j;
                o[0] = c_fma(o[0], tw, er);
                o[vs] = c_fma(o[vs], tw, ep);
                o[2 * vs] = c_fma(o[2 * vs], tw, ez);
            }
        }
        hp_km = hp;
        hr_km = hr;
    }
}


// access at a byte offset from a (wave-uniform) row base: the address is one
// scalar base pair plus a 32-bit lane offset
__device__ __forceinline__ float2 ldo(const float2 *row, unsigned off)
{
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(row) + off);
}
__device__ __forceinline__ const float2 *pco(const float2 *row, unsigned off)
{
    return reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(row) + off);
}
__device__ __forceinline__ float2 *pto(float2 *row, unsigned off)
{
    return reinterpret_cast<float2 *>(reinterpret_cast<char *>(row) + off);
}

// store of a value no block of this launch reads again (the next buffer set)
__device__ __forceinline__ void store_out(float2 *p, float2 v, bool nt)
{
    if (nt) {
        unsigned long long bits;
        __builtin_memcpy(&bits, &v, sizeof bits);
        __builtin_nontemporal_store(bits, reinterpret_cast<unsigned long long *>(p));
    } else {
        *p = v;
    }
}

// y = x / (1 + s F) reading the auxiliary from one buffer and, when the
// caller owns the cell, writing its update to the other
__device__ __forceinline__ float2 div_stretch2(float2 x, const float2 *src, float2 *dst, bool store, float g1,
                                               float g2, float c, float dt)
{
    float2 u = *src;
    float2 y = make_float2(g1 * x.x - g2 * u.x, g1 * x.y - g2 * u.y);
    if (store) *dst = make_float2(c * u.x + dt * y.x, c * u.y + dt * y.y);
    return y;
}

// Auxiliary row bases of one cell row for the recursions: r-layer slab row
// (k, ir) and z-layer slab row (kz, i) of one auxiliary set.  Slot q of a
// cell is the r-layer auxiliary q (q < N_AUX_R) or the z-layer auxiliary
// q - N_AUX_R.
struct AuxRows {
    const float2 *sR, *sZ;   // read (time level before the half-step)
    float2 *dR, *dZ;         // written (time level after it)
    __device__ __forceinline__ float2 ld(int q, size_t slabR, size_t slabZ, unsigned o) const
    {
        return q < N_AUX_R ? ldo(sR + q * slabR, o) : ldo(sZ + (q - N_AUX_R) * slabZ, o);
    }
    __device__ __forceinline__ void st(int q, float2 v, size_t slabR, size_t slabZ, unsigned o) const
    {
        *(q < N_AUX_R ? pto(dR + q * slabR, o) : pto(dZ + (q - N_AUX_R) * slabZ, o)) = v;
    }
};

// a cell's auxiliaries at one time level held in registers (slots as above)
constexpr int N_SLOT = N_AUX_R + N_AUX_Z;
struct AuxCarry {
    float2 v[N_SLOT];
};

// read from registers, write to memory (the level after the half-step)
struct AuxFromReg {
    const AuxCarry *r;
    float2 *dR, *dZ;
    __device__ __forceinline__ float2 ld(int q, size_t, size_t, unsigned) const { return r->v[q]; }
    __device__ __forceinline__ void st(int q, float2 v, size_t slabR, size_t slabZ, unsigned o) const
    {
        *(q < N_AUX_R ? pto(dR + q * slabR, o) : pto(dZ + (q - N_AUX_R) * slabZ, o)) = v;
    }
};

// read from registers loaded together beforehand (the level before the
// half-step), write to registers
struct AuxPreToReg {
    const AuxCarry *p;
    AuxCarry *r;
    __device__ __forceinline__ float2 ld(int q, size_t, size_t, unsigned) const { return p->v[q]; }
    __device__ __forceinline__ void st(int q, float2 v, size_t, size_t, unsigned) const { r->v[q] = v; }
};

// y = x / (1 + s F) with the auxiliary of slot q read through io and, when
// store, its update written through io
template <class X>
__device__ __forceinline__ float2 div_stretch_io(float2 x, const X &io, int q, size_t slabR, size_t slabZ, unsigned o,
                                                 bool store, float g1, float g2, float c, float dt)
{
    const float2 u = io.ld(q, slabR, slabZ, o);
    const float2 y = make_float2(g1 * x.x - g2 * u.x, g1 * x.y - g2 * u.y);
    if (store) io.st(q, make_float2(c * u.x + dt * y.x, c * u.y + dt * y.y), slabR, slabZ, o);
    return y;
}

// H half-step of one cell, H^{n+1/2} = H^{n-1/2} - dt curl E^n, with the PML
// divide-by-stretch recursions.  E^n at the cell and its +phi (jp), +r (ip)
// and +z (kp) neighbours; u0, u1 are U = F E_phi at rows i and i + 1 (r-layer
// only).  The auxiliaries of the cell are written when wr; v returns the
// updated V = F H_phi (r-layer; zero elsewhere).  Inner boundary (i = 0):
// H_r is not updated unless the row borders the axis; bottom plane (k = 0):
// H_z is not updated.
template <class X>
__device__ __forceinline__ void h_cell(const StepArgs &a, const RowCoef &rc, const ZCoef &zc, int i, int k, int ir,
                                       int kz, size_t slabR, size_t slabZ, const X &x, unsigned o, bool wr,
                                       float2 ez, float2 er, float2 ep, float2 ez_jp, float2 er_jp, float2 er_kp,
                                       float2 ep_kp, float2 ez_ip, float2 ep_ip, float2 u0, float2 u1, float2 &hr,
                                       float2 &hp, float2 &hz, float2 &v)
{
    const float dt = a.dt;
    // H_r at (i, j+1/2, k+1/2)
    if (i > 0 || a.axis) {
        float2 t1 = c_scale(c_sub(ez_jp, ez), rc.inv_rdphi_int);
        float2 t2 = c_scale(c_sub(ep_kp, ep), a.inv_dz);
        if (ir >= 0)
            t1 = div_stretch_io(t1, x, AUX_HR_T, slabR, slabZ, o, wr,
                              rc.g1_t_int, rc.g2_t_int, a.cr, dt);
        if (kz >= 0)
            t2 = div_stretch_io(t2, x, N_AUX_R + ZAUX_HR, slabR, slabZ, o, wr, zc.g1_half,
                              zc.g2_half, a.cz, dt);
        hr = make_float2(hr.x - dt * (t1.x - t2.x), hr.y - dt * (t1.y - t2.y));
    }
    // H_phi at (i+1/2, j, k+1/2)
    {
        float2 t1 = c_scale(c_sub(er_kp, er), a.inv_dz);
        float2 t2 = c_scale(c_sub(ez_ip, ez), a.inv_dr);
        if (kz >= 0)
            t1 = div_stretch_io(t1, x, N_AUX_R + ZAUX_HP, slabR, slabZ, o, wr, zc.g1_half,
                              zc.g2_half, a.cz, dt);
        if (ir >= 0)
            t2 = div_stretch_io(t2, x, AUX_HP_S, slabR, slabZ, o, wr,
                              rc.g1_s_half, rc.g2_s_half, a.cr, dt);
        hp = make_float2(hp.x - dt * (t1.x - t2.x), hp.y - dt * (t1.y - t2.y));
        v = zero2();
        if (ir >= 0) {
            const float2 vo = x.ld(AUX_V_HP, slabR, slabZ, o);
            v = make_float2(a.cr * vo.x + dt * hp.x, a.cr * vo.y + dt * hp.y);
            if (wr) x.st(AUX_V_HP, v, slabR, slabZ, o);
        }
    }
    // H_z at (i+1/2, j+1/2, k)
    if (k > 0) {
        float2 t = c_add(c_scale(c_sub(ep_ip, ep), a.inv_dr), c_scale(c_add(ep_ip, ep), rc.inv_2r_half));
        if (ir >= 0) {
            t = c_add(t, c_sub(c_scale(u1, rc.hz_c1), c_scale(u0, rc.hz_c0)));
            t = div_stretch_io(t, x, AUX_HZ_S, slabR, slabZ, o, wr, rc.g1_s_half,
                             rc.g2_s_half, a.cr, dt);
        }
        t = c_sub(t, c_scale(c_sub(er_jp, er), rc.inv_rdphi_half));
        if (ir >= 0)
            t = div_stretch_io(t, x, AUX_HZ_T, slabR, slabZ, o, wr, rc.g1_t_half,
                             rc.g2_t_half, a.cr, dt);
        hz = make_float2(hz.x - dt * t.x, hz.y - dt * t.y);
    }
}

// E half-step of one cell, E^{n+1} = E^n + (dt/eps)(curl H^{n+1/2} - J), with
// the PML recursions.  H^{n+1/2} at the cell and its -phi (jm), -r (im) and
// -z (km) neighbours, V at rows i and i - 1, the source current (jr, jph).
// The auxiliaries are always written (only owners call it with a write
// target); u returns the updated U = F E_phi (r-layer, every cell).  Inner
// boundary: E_phi and E_z are not updated, except next to the axis, where the
// -r neighbours (H_z on the axis, H_phi at r = 0) count as zero whatever the
// caller passes; bottom plane: E_r and E_phi are not updated.
template <class X>
__device__ __forceinline__ void e_cell(const StepArgs &a, const RowCoef &rc, const ZCoef &zc, int i, int k, int ir,
                                       int kz, size_t slabR, size_t slabZ, const X &x, unsigned o, float ce,
                                       float2 jr, float2 jph, float2 hr, float2 hr_jm, float2 hr_km, float2 hp,
                                       float2 hp_im, float2 hp_km, float2 hz, float2 hz_jm, float2 hz_im, float2 v,
                                       float2 v_im, float2 &er, float2 &ep, float2 &ez, float2 &u)
{
    const float dt = a.dt;
    if (i == 0) { hz_im = zero2(); hp_im = zero2(); v_im = zero2(); }
    // E_r at (i+1/2, j, k)
    if (k > 0) {
        float2 t1 = c_scale(c_sub(hz, hz_jm), rc.inv_rdphi_half);
        float2 t2 = c_scale(c_sub(hp, hp_km), a.inv_dz);
        if (ir >= 0)
            t1 = div_stretch_io(t1, x, AUX_ER_T, slabR, slabZ, o, true,
                              rc.g1_t_half, rc.g2_t_half, a.cr, dt);
        if (kz >= 0)
            t2 = div_stretch_io(t2, x, N_AUX_R + ZAUX_ER, slabR, slabZ, o, true, zc.g1_int,
                              zc.g2_int, a.cz, dt);
        er = make_float2(er.x + ce * (t1.x - t2.x - jr.x), er.y + ce * (t1.y - t2.y - jr.y));
    }
    // E_phi at (i, j+1/2, k)
    u = zero2();
    if (k > 0 && (i > 0 || a.axis)) {
        float2 t1 = c_scale(c_sub(hr, hr_km), a.inv_dz);
        float2 t2 = c_scale(c_sub(hz, hz_im), a.inv_dr);
        if (kz >= 0)
            t1 = div_stretch_io(t1, x, N_AUX_R + ZAUX_EP, slabR, slabZ, o, true, zc.g1_int,
                              zc.g2_int, a.cz, dt);
        if (ir >= 0)
            t2 = div_stretch_io(t2, x, AUX_EP_S, slabR, slabZ, o, true,
                              rc.g1_s_int, rc.g2_s_int, a.cr, dt);
        ep = make_float2(ep.x + ce * (t1.x - t2.x - jph.x), ep.y + ce * (t1.y - t2.y - jph.y));
    }
    // U = F E_phi advances on every r-layer cell (also where E_phi is held)
    if (ir >= 0) {
        const float2 uo = x.ld(AUX_U_EP, slabR, slabZ, o);
        u = make_float2(a.cr * uo.x + dt * ep.x, a.cr * uo.y + dt * ep.y);
        x.st(AUX_U_EP, u, slabR, slabZ, o);
    }
    // E_z at (i, j, k+1/2)
    if (i > 0 || a.axis) {
        float2 t = c_add(c_scale(c_sub(hp, hp_im), a.inv_dr), c_scale(c_add(hp, hp_im), rc.inv_2r_int));
        if (ir >= 0) {
            t = c_add(t, c_sub(c_scale(v, rc.ez_c1), c_scale(v_im, rc.ez_c0)));
            t = div_stretch_io(t, x, AUX_EZ_S, slabR, slabZ, o, true,
                             rc.g1_s_int, rc.g2_s_int, a.cr, dt);
        }
        t = c_sub(t, c_scale(c_sub(hr, hr_jm), rc.inv_rdphi_int));
        if (ir >= 0)
            t = div_stretch_io(t, x, AUX_EZ_T, slabR, slabZ, o, true,
                             rc.g1_t_int, rc.g2_t_int, a.cr, dt);
        ez = make_float2(ez.x + ce * t.x, ez.y + ce * t.y);
    }
}

// Source current of the sheet at plane k_src for step n at one cell.
__device__ __forceinline__ void sheet_current(const StepArgs &a, int n, size_t plane, size_t rowc, unsigned o,
                                              float2 &jr, float2 &jph)
{
    jr = zero2();
    jph = zero2();
    for (int q = 0; q < a.n_prof; ++q) {
        const float2 g = a.profile[(size_t)n * a.n_prof + q];
        const float2 *pat = a.pattern + (size_t)q * 2 * plane + rowc;
        jr = c_fma(jr, ldo(pat, o), g);
        jph = c_fma(jph, ldo(pat + plane, o), g);
    }
}

// One whole leap-frog step (H half-step, then E half-step with source and
// DFT) per launch, reading fields and auxiliaries from one buffer set and
// writing the next time level to the other, so no block ever reads a value
// another block of the same launch writes.  Block = (TR + 1) wavefronts x 64
// lanes marching a z-chunk: wave 0 recomputes H on the radial halo row
// i0 - 1, waves 1..TR own rows i0 .. i0 + TR - 1; lane l sits on phi cell
// j0 - 1 + l (j0 = FUSED_COLS x tile column), lane 0 recomputes H on the
// azimuthal halo column (across the wedge seam for the first tile), lanes
// 1..FUSED_COLS own (the lanes above compute cells they do not store).  Each
// plane's H^{n+1/2} goes through LDS (two buffers, one barrier per plane) to
// the owners' E half-step.  A chunk starts one plane early to rebuild
// H^{n+1/2} at k = kb - 1 for the E half-step at kb.
template <int TR>
__device__ __forceinline__ void eh_fused_body(const StepArgs &a, int n, unsigned p, unsigned gx, unsigned gy)
{
    __shared__ float2 sHz[2][TR + 1][64], sHr[2][TR + 1][64], sHp[2][TR + 1][64], sV[2][TR + 1][64];
    const int lane = threadIdx.x;
    // a wavefront works on one row: the row index, its coefficients and every
    // row base address are wave-uniform (scalar registers); a lane only
    // carries its byte offset within the row
    const int ww = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    const int bx = (int)(p % gx), by = (int)((p / gx) % gy), bz = (int)(p / (gx * gy));
    const int i = by * TR + ww - 1;
    const bool row_ok = i >= 0 && i < nr;
    const int jj = bx * FUSED_COLS - 1 + lane;
    const bool hval = row_ok && jj < nphi;
    const bool seam_lane = jj < 0;
    const int j = seam_lane ? nphi - 1 : jj;
    const bool owner = ww >= 1 && lane >= 1 && lane <= FUSED_COLS && hval;
    const int kb = bz * a.kchunk;
    const int ke = min(kb + a.kchunk, nz);
    const int kstart = kb > 0 ? kb - 1 : kb;
    const bool nt = a.nt_stores;
    const int ir = row_ok ? slab_row(i, nr, a.pr0, a.pr1) : -1;
    const int ir1 = (row_ok && i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoef rc = a.rows[row_ok ? i : 0];
    // every field load is issued unconditionally (from a clamped row, column
    // or plane where the neighbour lies outside) so that a plane's loads are
    // all in flight together; out-of-range values are replaced afterwards
    const int ic = min(max(i, 0), nr - 1);
    const int jc = min(j, nphi - 1);
    const bool wrap = (jc + 1 >= nphi);
    const unsigned o = (unsigned)jc * 8u;             // complex sample j of a row
    const unsigned ojp = wrap ? 0u : o + 8u;         // sample j + 1 (column 0 across the seam)
    const unsigned oc = (unsigned)jc * 4u;            // real sample j of a row
    const size_t rowc = (size_t)ic * nphi;
    const bool ip_ok = ic + 1 < nr;
    const size_t dip = ip_ok ? (size_t)nphi : 0;
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const int nd = a.k1 - a.k0;

    float2 er = ldo(a.Er + (size_t)kstart * plane + rowc, o);
    float2 ep = ldo(a.Ep + (size_t)kstart * plane + rowc, o);
    float2 hr_km = zero2(), hp_km = zero2();
    for (int k = kstart; k < ke; ++k) {
        const size_t c0 = (size_t)k * plane + rowc;
        const bool kp_ok = k + 1 < nz;
        const size_t dkp = kp_ok ? plane : 0;
        const bool store = owner && k >= kb;
        const int kz = slab_row(k, nz, a.pz0, a.pz1);
        ZCoef zc = {};
        if (kz >= 0) zc = a.zrows[k];
        const size_t sr0 = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi : 0;
        const size_t sz0 = kz >= 0 ? ((size_t)kz * nr + ic) * nphi : 0;
        const AuxRows x = {a.auxR + sr0, a.auxZ + sz0, a.oauxR + sr0, a.oauxZ + sz0};
        const float2 ez = ldo(a.Ez + c0, o);
        float2 er_kp = ldo(a.Er + c0 + dkp, o), ep_kp = ldo(a.Ep + c0 + dkp, o);
        float2 ez_jp = ldo(a.Ez + c0, ojp), er_jp = ldo(a.Er + c0, ojp);
        float2 ez_ip = ldo(a.Ez + c0 + dip, o), ep_ip = ldo(a.Ep + c0 + dip, o);
        float2 hr = ldo(a.Hr + c0, o), hp = ldo(a.Hp + c0, o), hz = ldo(a.Hz + c0, o);
        float2 v = zero2();
        if (!kp_ok) { er_kp = zero2(); ep_kp = zero2(); }
        if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
        if (wrap) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
        {
            float2 u0 = zero2(), u1 = zero2();
            if (ir >= 0 && k > 0) {
                u0 = ldo(x.sR + AUX_U_EP * slabR, o);
                if (ir1 >= 0) u1 = ldo(a.auxR + AUX_U_EP * slabR + ((size_t)k * a.dR + ir1) * nphi, o);
            }
            h_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x, o, store, ez, er, ep, ez_jp, er_jp, er_kp, ep_kp, ez_ip,
                   ep_ip, u0, u1, hr, hp, hz, v);
            if (store) {
                store_out(pto(a.oHr + c0, o), hr, nt);
                store_out(pto(a.oHp + c0, o), hp, nt);
                store_out(pto(a.oHz + c0, o), hz, nt);
            }
        }
        if (!hval) { hr = zero2(); hp = zero2(); hz = zero2(); v = zero2(); }
        const int buf = k & 1;
        if (seam_lane) {   // the halo column across the wedge boundary is j = -1
            sHz[buf][ww][lane] = c_mul(a.seam_m, hz);
            sHr[buf][ww][lane] = c_mul(a.seam_m, hr);
            sHp[buf][ww][lane] = c_mul(a.seam_m, hp);
            sV[buf][ww][lane] = c_mul(a.seam_m, v);
        } else {
            sHz[buf][ww][lane] = hz;
            sHr[buf][ww][lane] = hr;
            sHp[buf][ww][lane] = hp;
            sV[buf][ww][lane] = v;
        }
        __syncthreads();
        if (store) {
            const float2 hz_jm = sHz[buf][ww][lane - 1], hr_jm = sHr[buf][ww][lane - 1];
            const float2 hz_im = sHz[buf][ww - 1][lane], hp_im = sHp[buf][ww - 1][lane];
            const float2 v_im = sV[buf][ww - 1][lane];
            const float ce = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a.ceps + c0) + oc);
            float2 jr = zero2(), jph = zero2();
            if (k == a.k_src) sheet_current(a, n, plane, rowc, o, jr, jph);
            float2 er_n = er, ep_n = ep, ez_n = ez, u;
            e_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x, o, ce, jr, jph, hr, hr_jm, hr_km, hp, hp_im, hp_km, hz,
                   hz_jm, hz_im, v, v_im, er_n, ep_n, ez_n, u);
            store_out(pto(a.oEr + c0, o), er_n, nt);
            store_out(pto(a.oEp + c0, o), ep_n, nt);
            store_out(pto(a.oEz + c0, o), ez_n, nt);
            if (a.dft_plane && k == a.k_mon) {
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw = a.twiddle[(size_t)n * a.K + f];
                    float2 *q0 = pto(a.dft_plane + (size_t)f * 2 * plane + rowc, o);
                    float2 *q1 = pto(a.dft_plane + (size_t)f * 2 * plane + plane + rowc, o);
                    *q0 = c_fma(*q0, tw, er_n);
                    *q1 = c_fma(*q1, tw, ep_n);
                }
            }
            if (a.dft_vol && k >= a.k0 && k < a.k1) {
                const size_t vs = (size_t)nd * plane;
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw = a.twiddle[(size_t)n * a.K + f];
                    float2 *base = a.dft_vol + (size_t)f * 3 * vs + (size_t)(k - a.k0) * plane + rowc;
                    float2 *q0 = pto(base, o), *q1 = pto(base + vs, o), *q2 = pto(base + 2 * vs, o);
                    *q0 = c_fma(*q0, tw, er_n);
                    *q1 = c_fma(*q1, tw, ep_n);
                    *q2 = c_fma(*q2, tw, ez_n);
                }
            }
        }
        hr_km = hr;
        hp_km = hp;
        er = er_kp;
        ep = ep_kp;
    }
}

// One whole leap-frog step with the flat (r, phi) mapping, for narrow wedges:
// a block of FLAT_BLOCK threads holds R = FLAT_BLOCK / nphi - 1 whole rows
// i0 .. i0 + R - 1 plus the halo row i0 - 1 below them, thread t on row
// i0 - 1 + t / nphi, column t % nphi.  Every thread computes H^{n+1/2} of its
// cell from E^n (global loads; the +phi neighbour of the last column is
// column 0 times the seam factor); H goes through LDS to the E half-step of
// the owned rows, whose -phi neighbour of column 0 is the row's last column
// times the inverse seam factor and whose -r neighbour is one row (nphi
// threads) back.  Reads set A, writes set B; one barrier per plane.
__device__ __forceinline__ void eh_flat_body(const StepArgs &a, int n, unsigned brow, unsigned bz)
{
    __shared__ float2 sHz[2][FLAT_BLOCK], sHr[2][FLAT_BLOCK], sHp[2][FLAT_BLOCK], sV[2][FLAT_BLOCK];
    const int t = threadIdx.x;
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const int R = FLAT_BLOCK / nphi - 1;                // owned rows per block
    const size_t plane = (size_t)nr * nphi;
    const int ri = t / nphi, j = t - ri * nphi;         // ri = 0: the halo row
    const int i = (int)brow * R - 1 + ri;
    const bool in_block = ri <= R;
    const bool row_ok = in_block && i >= 0 && i < nr;
    const bool owner = row_ok && ri >= 1;
    const int kb = (int)bz * a.kchunk;
    const int ke = min(kb + a.kchunk, nz);
    const int kstart = kb > 0 ? kb - 1 : kb;
    const bool nt = a.nt_stores;
    const int ir = row_ok ? slab_row(i, nr, a.pr0, a.pr1) : -1;
    const int ir1 = (row_ok && i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoef rc = a.rows[row_ok ? i : 0];
    const int ic = min(max(i, 0), nr - 1);
    const bool wrap = j + 1 >= nphi;
    const unsigned o = (unsigned)j * 8u;
    const unsigned ojp = wrap ? 0u : o + 8u;
    const unsigned oc = (unsigned)j * 4u;
    const size_t rowc = (size_t)ic * nphi;
    const bool ip_ok = ic + 1 < nr;
    const size_t dip = ip_ok ? (size_t)nphi : 0;
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const int nd = a.k1 - a.k0;
    // LDS slots of the -phi neighbour (the row's last column across the seam)
    // and of the -r neighbour
    const int t_jm = j > 0 ? t - 1 : t + nphi - 1;
    const int t_im = t >= nphi ? t - nphi : t;

    float2 er = ldo(a.Er + (size_t)kstart * plane + rowc, o);
    float2 ep = ldo(a.Ep + (size_t)kstart * plane + rowc, o);
    float2 hr_km = zero2(), hp_km = zero2();
    for (int k = kstart; k < ke; ++k) {
        const size_t c0 = (size_t)k * plane + rowc;
        const bool kp_ok = k + 1 < nz;
        const size_t dkp = kp_ok ? plane : 0;
        const bool store = owner && k >= kb;
        const int kz = slab_row(k, nz, a.pz0, a.pz1);
        ZCoef zc = {};
        if (kz >= 0) zc = a.zrows[k];
        const size_t sr0 = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi : 0;
        const size_t sz0 = kz >= 0 ? ((size_t)kz * nr + ic) * nphi : 0;
        const AuxRows x = {a.auxR + sr0, a.auxZ + sz0, a.oauxR + sr0, a.oauxZ + sz0};
        const float2 ez = ldo(a.Ez + c0, o);
        float2 er_kp = ldo(a.Er + c0 + dkp, o), ep_kp = ldo(a.Ep + c0 + dkp, o);
        float2 ez_jp = ldo(a.Ez + c0, ojp), er_jp = ldo(a.Er + c0, ojp);
        float2 ez_ip = ldo(a.Ez + c0 + dip, o), ep_ip = ldo(a.Ep + c0 + dip, o);
        float2 hr = ldo(a.Hr + c0, o), hp = ldo(a.Hp + c0, o), hz = ldo(a.Hz + c0, o);
        float2 v = zero2();
        if (!kp_ok) { er_kp = zero2(); ep_kp = zero2(); }
        if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
        if (wrap) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
        {
            float2 u0 = zero2(), u1 = zero2();
            if (ir >= 0 && k > 0) {
                u0 = ldo(x.sR + AUX_U_EP * slabR, o);
                if (ir1 >= 0) u1 = ldo(a.auxR + AUX_U_EP * slabR + ((size_t)k * a.dR + ir1) * nphi, o);
            }
            h_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x, o, store, ez, er, ep, ez_jp, er_jp, er_kp, ep_kp, ez_ip,
                   ep_ip, u0, u1, hr, hp, hz, v);
            if (store) {
                store_out(pto(a.oHr + c0, o), hr, nt);
                store_out(pto(a.oHp + c0, o), hp, nt);
                store_out(pto(a.oHz + c0, o), hz, nt);
            }
        }
        if (!row_ok) { hr = zero2(); hp = zero2(); hz = zero2(); v = zero2(); }
        const int buf = k & 1;
        sHz[buf][t] = hz;
        sHr[buf][t] = hr;
        sHp[buf][t] = hp;
        sV[buf][t] = v;
        __syncthreads();
        if (store) {
            float2 hz_jm = sHz[buf][t_jm], hr_jm = sHr[buf][t_jm];
            if (j == 0) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
            const float2 hz_im = sHz[buf][t_im], hp_im = sHp[buf][t_im];
            const float2 v_im = sV[buf][t_im];
            const float ce = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a.ceps + c0) + oc);
            float2 jr = zero2(), jph = zero2();
            if (k == a.k_src) sheet_current(a, n, plane, rowc, o, jr, jph);
            float2 er_n = er, ep_n = ep, ez_n = ez, u;
            e_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x, o, ce, jr, jph, hr, hr_jm, hr_km, hp, hp_im, hp_km, hz,
                   hz_jm, hz_im, v, v_im, er_n, ep_n, ez_n, u);
            store_out(pto(a.oEr + c0, o), er_n, nt);
            store_out(pto(a.oEp + c0, o), ep_n, nt);
            store_out(pto(a.oEz + c0, o), ez_n, nt);
            if (a.dft_plane && k == a.k_mon) {
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw = a.twiddle[(size_t)n * a.K + f];
                    float2 *q0 = pto(a.dft_plane + (size_t)f * 2 * plane + rowc, o);
                    float2 *q1 = pto(a.dft_plane + (size_t)f * 2 * plane + plane + rowc, o);
                    *q0 = c_fma(*q0, tw, er_n);
                    *q1 = c_fma(*q1, tw, ep_n);
                }
            }
            if (a.dft_vol && k >= a.k0 && k < a.k1) {
                const size_t vs = (size_t)nd * plane;
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw = a.twiddle[(size_t)n * a.K + f];
                    float2 *base = a.dft_vol + (size_t)f * 3 * vs + (size_t)(k - a.k0) * plane + rowc;
                    float2 *q0 = pto(base, o), *q1 = pto(base + vs, o), *q2 = pto(base + 2 * vs, o);
                    *q0 = c_fma(*q0, tw, er_n);
                    *q1 = c_fma(*q1, tw, ep_n);
                    *q2 = c_fma(*q2, tw, ez_n);
                }
            }
        }
        hr_km = hr;
        hp_km = hp;
        er = er_kp;
        ep = ep_kp;
    }
}

// Field values one cell's step-one H half-step reads at plane k (plus dt/eps
// at k), loaded unconditionally from in-range addresses: the +z neighbour is
// plane k + 1 (plane k itself at the top), the +r neighbour row ic + dip.
struct PlaneIn {
    float2 ez, er_kp, ep_kp, ez_jp, er_jp, ez_ip, ep_ip, hr, hp, hz;
    float ce;
};

__device__ __forceinline__ PlaneIn load_plane(const StepArgs &a, int k, size_t plane, size_t rowc, size_t dip,
                                              unsigned o, unsigned ojp, unsigned oc)
{
    const size_t c0 = (size_t)k * plane + rowc;
    const size_t dkp = k + 1 < a.nz ? plane : 0;
    PlaneIn p;
    p.ez = ldo(a.Ez + c0, o);
    p.er_kp = ldo(a.Er + c0 + dkp, o);
    p.ep_kp = ldo(a.Ep + c0 + dkp, o);
    p.ez_jp = ldo(a.Ez + c0, ojp);
    p.er_jp = ldo(a.Er + c0, ojp);
    p.ez_ip = ldo(a.Ez + c0 + dip, o);
    p.ep_ip = ldo(a.Ep + c0 + dip, o);
    p.hr = ldo(a.Hr + c0, o);
    p.hp = ldo(a.Hp + c0, o);
    p.hz = ldo(a.Hz + c0, o);
    p.ce = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a.ceps + c0) + oc);
    return p;
}

// Two whole leap-frog steps (n and n + 1) per launch.  The launch reads the
// fields and auxiliaries at time level n from one buffer set and writes level
// n + 2 to the other, so each cell's six fields cross HBM once per two steps.
// Block = (TR + 3) wavefronts x 64 lanes marching a z-chunk: wave w sits on
// row i0 - 2 + w and lane l on phi cell j0 - 2 + l (j0 = COLS x tile column,
// COLS = two_step_cols(LAY)),
// taken modulo nphi (physical cells; the Bloch seam factor is applied where a
// neighbour value crosses from column nphi - 1 to 0).  Step one runs on every
// lane and wave; its H^{n+1/2} reaches the E half-step through LDS.  Step two
// lags one plane behind and needs E^{n+1} of the +phi, +r neighbours
// (double-buffered LDS) and H^{n+3/2} of the -phi, -r neighbours (LDS); it
// is exact on lanes 2..62 and waves 2..nrow+1 (nrow <= TR owned rows); lanes
// 2..COLS+1 of those waves own their cells.  A chunk
// starts two planes early and runs step one one plane past its end.  Every
// block computes halo cells with the same inputs and the same arithmetic as
// their owner, so the level-(n+1) auxiliaries that step one writes to the
// intermediate set are identical whichever block writes them.
//
// CARRY: the level-(n+1) auxiliaries stay in registers from step one at
// plane k to step two at the same plane (the next iteration) instead of
// going through the intermediate set: each thread reads back only what it
// wrote itself, so the values and the arithmetic are the same.  The level-n
// auxiliaries that step one reads are loaded together at the start of the
// plane, so their latencies overlap.  It costs three sets of the cell's
// auxiliaries in registers, which the layer tiles of a narrower block (or
// with the z-layer recursions only) can hold.
template <int TR, int LAY, bool CARRY = false>
__device__ __forceinline__ void eh2_body(const StepArgs &a, int n, uint4 tile)
{
    // LAY bit 0: the tile's rows include r-layer rows; bit 1: its planes include z-layer planes
    constexpr bool PR = (LAY & 1) != 0, PZ = (LAY & 2) != 0;
    constexpr int NW = TR + 3;
    constexpr int NV = PR ? NW : 1;
    __shared__ float2 s1z[NW][64], s1r[NW][64], s1p[NW][64], s1v[NV][64];
    __shared__ float2 sEz[2][NW][64], sEr[2][NW][64], sEp[2][NW][64], sU[2][NV][64];
    __shared__ float2 s2z[NW][64], s2r[NW][64], s2p[NW][64], s2v[NV][64];
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    // tile: phi column block, first owned row and row count (<= TR), planes [kb, ke)
    const int bx = (int)tile.x, i0 = (int)(tile.y & 0xffffu), nrow = (int)(tile.y >> 16);
    const int kb = (int)(tile.z & 0xffffu), ke = (int)(tile.z >> 16);
    const int i = i0 + w - 2;
    const bool active = w <= nrow + 2;                      // waves above the top halo row idle
    const bool row_ok = active && i >= 0 && i < nr;
    constexpr int COLS = two_step_cols(LAY);
    const int jj = bx * COLS - 2 + lane;
    const int pc = (jj + nphi) % nphi;                      // physical column
    const bool cross_m = pc == 0;                           // lane - 1 holds column nphi - 1
    const bool cross_p = pc == nphi - 1;                    // lane + 1 holds column 0
    const bool own = lane >= 2 && lane < 2 + COLS && jj < nphi && w >= 2 && w <= nrow + 1 && row_ok;
    const int k_lo = max(kb - 2, 0);
    const bool nt = a.nt_stores;
    const int ir = (PR && row_ok) ? slab_row(i, nr, a.pr0, a.pr1) : -1;
    const int ir1 = (PR && row_ok && i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoef rc = a.rows[row_ok ? i : 0];
    const int ic = min(max(i, 0), nr - 1);
    const unsigned o = (unsigned)pc * 8u;
    const unsigned ojp = cross_p ? 0u : o + 8u;
    const unsigned oc = (unsigned)pc * 4u;
    const size_t rowc = (size_t)ic * nphi;
    const bool ip_ok = ic + 1 < nr;
    const size_t dip = ip_ok ? (size_t)nphi : 0;
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const int nd = a.k1 - a.k0;

    // carried along z: E^n at k; H^{n+1/2}, E^{n+1}, U^{n+1}, dt/eps at k - 1;
    // H^{n+3/2} at k - 2
    float2 er0 = ldo(a.Er + (size_t)k_lo * plane + rowc, o);
    float2 ep0 = ldo(a.Ep + (size_t)k_lo * plane + rowc, o);
    float2 h1r_p = zero2(), h1p_p = zero2(), h1z_p = zero2();
    float2 e1r_p = zero2(), e1p_p = zero2(), e1z_p = zero2(), u1_p = zero2();
    float2 h2r_km = zero2(), h2p_km = zero2();
    float ce_p = 0.f;
    // the next plane's loads are issued one plane ahead (where the registers
    // allow), so they are in flight through this plane's barriers and updates
    constexpr bool PF = !PR && !CARRY;
    using X1 = std::conditional_t<CARRY, AuxPreToReg, AuxRows>;
    using X2 = std::conditional_t<CARRY, AuxFromReg, AuxRows>;
    AuxCarry car_c, car_p;   // CARRY: step one's auxiliaries of planes k and k - 1
    AuxCarry pre;            // CARRY: the level-n auxiliaries of plane k, all loads issued together
    PlaneIn cur = load_plane(a, k_lo, plane, rowc, dip, o, ojp, oc);
    for (int k = k_lo; k <= ke; ++k) {
        const int km = k - 1;
        PlaneIn in;
        if (!PF) {
            in = load_plane(a, min(k, nz - 1), plane, rowc, dip, o, ojp, oc);
        } else {
            in = cur;
            cur = load_plane(a, min(k + 1, min(ke, nz - 1)), plane, rowc, dip, o, ojp, oc);
        }
        float2 h1r = zero2(), h1p = zero2(), h1z = zero2(), v1 = zero2();
        float2 e1r = zero2(), e1p = zero2(), e1z = zero2(), u1 = zero2();
        float2 er_kp = zero2(), ep_kp = zero2();
        float ce = 0.f;
        const bool step1 = k < nz;
        // ---- step one, H^{n+1/2} at plane k (every lane and wave)
        int kz = -1;
        ZCoef zc = {};
        X1 x1 = {};
        if constexpr (CARRY) x1.r = &car_c;   // set on every path, so the carry stays in registers
        if constexpr (CARRY) x1.p = &pre;
        float2 ez0 = zero2();
        if (step1 && active) {
            kz = PZ ? slab_row(k, nz, a.pz0, a.pz1) : -1;
            if (kz >= 0) zc = a.zrows[k];
            const size_t sr0 = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi : 0;
            const size_t sz0 = kz >= 0 ? ((size_t)kz * nr + ic) * nphi : 0;
            if constexpr (CARRY) {
                if (ir >= 0)
                    for (int q = 0; q < N_AUX_R; ++q) pre.v[q] = ldo(a.auxR + sr0 + q * slabR, o);
                if (kz >= 0)
                    for (int q = 0; q < N_AUX_Z; ++q) pre.v[N_AUX_R + q] = ldo(a.auxZ + sz0 + q * slabZ, o);
            } else {
                x1.sR = a.auxR + sr0;
                x1.sZ = a.auxZ + sz0;
            }
            if constexpr (!CARRY) {
                x1.dR = a.mauxR + sr0;
                x1.dZ = a.mauxZ + sz0;
            }
            const bool kp_ok = k + 1 < nz;
            ez0 = in.ez;
            er_kp = in.er_kp;
            ep_kp = in.ep_kp;
            float2 ez_jp = in.ez_jp, er_jp = in.er_jp;
            float2 ez_ip = in.ez_ip, ep_ip = in.ep_ip;
            h1r = in.hr;
            h1p = in.hp;
            h1z = in.hz;
            ce = in.ce;
            if (!kp_ok) { er_kp = zero2(); ep_kp = zero2(); }
            if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
            if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
            float2 u0 = zero2(), uu1 = zero2();
            if (ir >= 0 && k > 0) {
                if constexpr (CARRY) u0 = pre.v[AUX_U_EP];
                else u0 = ldo(a.auxR + sr0 + AUX_U_EP * slabR, o);
                if (ir1 >= 0) uu1 = ldo(a.auxR + AUX_U_EP * slabR + ((size_t)k * a.dR + ir1) * nphi, o);
            }
            h_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, row_ok, ez0, er0, ep0, ez_jp, er_jp, er_kp, ep_kp,
                   ez_ip, ep_ip, u0, uu1, h1r, h1p, h1z, v1);
            s1z[w][lane] = h1z;
            s1r[w][lane] = h1r;
            s1p[w][lane] = h1p;
            if (PR) s1v[w][lane] = v1;
        }
        __syncthreads();
        // ---- step one, E^{n+1} at plane k (exact on lanes >= 1, waves >= 1)
        if (step1 && (k != k_lo || k == 0) && w >= 1 && row_ok) {
            // lane 0's E^{n+1} feeds no owned cell; without layer recursions
            // (no auxiliary stores) it is computed like the others, from a
            // clamped neighbour, so the half-step runs without a lane mask
            if (!PR && !PZ || lane >= 1) {
                const int lm = lane > 0 ? lane - 1 : 0;
                float2 hz_jm = s1z[w][lm], hr_jm = s1r[w][lm];
                if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
                const float2 hz_im = s1z[w - 1][lane], hp_im = s1p[w - 1][lane];
                const float2 v_im = PR ? s1v[PR ? w - 1 : 0][lane] : zero2();
                float2 jr = zero2(), jph = zero2();
                if (k == a.k_src) sheet_current(a, n, plane, rowc, o, jr, jph);
                e1r = er0;
                e1p = ep0;
                e1z = ez0;
                e_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, ce, jr, jph, h1r, hr_jm, h1r_p, h1p, hp_im,
                       h1p_p, h1z, hz_jm, hz_im, v1, v_im, e1r, e1p, e1z, u1);
            }
            sEz[k & 1][w][lane] = e1z;
            sEr[k & 1][w][lane] = e1r;
            sEp[k & 1][w][lane] = e1p;
            if (PR) sU[k & 1][PR ? w : 0][lane] = u1;
        }
        // ---- step two, H^{n+3/2} at plane km (exact on lanes 1..62, waves 1..TR+1)
        float2 h2r = zero2(), h2p = zero2(), h2z = zero2(), v2 = zero2();
        const bool h2_plane = km >= 0 && (km > k_lo || km == 0);
        const int kz2 = (PZ && km >= 0) ? slab_row(km, nz, a.pz0, a.pz1) : -1;
        ZCoef zc2 = {};
        if (kz2 >= 0) zc2 = a.zrows[km];
        const size_t c0m = (size_t)max(km, 0) * plane + rowc;
        const size_t sr2 = ir >= 0 ? ((size_t)max(km, 0) * a.dR + ir) * nphi : 0;
        const size_t sz2 = kz2 >= 0 ? ((size_t)kz2 * nr + ic) * nphi : 0;
        X2 x2;
        if constexpr (CARRY) x2 = X2{&car_p, a.oauxR + sr2, a.oauxZ + sz2};
        else x2 = X2{a.mauxR + sr2, a.mauxZ + sz2, a.oauxR + sr2, a.oauxZ + sz2};
        const bool store = own && km >= kb && km < ke;
        // lanes 0 and 63 feed no owned cell: without layer recursions they
        // compute from clamped neighbours instead of being masked off
        if (h2_plane && w >= 1 && w <= nrow + 1 && row_ok && (!PR && !PZ || (lane >= 1 && lane <= 62))) {
            const int b = km & 1;
            const int lp = lane < 63 ? lane + 1 : 63;
            float2 ez_jp = sEz[b][w][lp], er_jp = sEr[b][w][lp];
            if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
            float2 ez_ip = sEz[b][w + 1][lane], ep_ip = sEp[b][w + 1][lane];
            if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
            float2 uu1 = zero2();
            if (PR && ir1 >= 0) uu1 = sU[b][PR ? w + 1 : 0][lane];
            h2r = h1r_p;
            h2p = h1p_p;
            h2z = h1z_p;
            // E^{n+1} at km + 1 is the plane step one just finished (zero above the top)
            h_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, store, e1z_p, e1r_p, e1p_p, ez_jp, er_jp, e1r,
                   e1p, ez_ip, ep_ip, (ir >= 0 && km > 0) ? u1_p : zero2(), uu1, h2r, h2p, h2z, v2);
        }
        s2z[w][lane] = h2z;
        s2r[w][lane] = h2r;
        s2p[w][lane] = h2p;
        if (PR) s2v[w][lane] = v2;
        __syncthreads();
        // ---- step two, E^{n+2} at plane km (owners), stores and DFT
        if (store) {
            float2 hz_jm = s2z[w][lane - 1], hr_jm = s2r[w][lane - 1];
            if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
            const float2 hz_im = s2z[w - 1][lane], hp_im = s2p[w - 1][lane];
            const float2 v_im = PR ? s2v[PR ? w - 1 : 0][lane] : zero2();
            float2 jr = zero2(), jph = zero2();
            if (km == a.k_src) sheet_current(a, n + 1, plane, rowc, o, jr, jph);
            float2 er2 = e1r_p, ep2 = e1p_p, ez2 = e1z_p, u2;
            e_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, ce_p, jr, jph, h2r, hr_jm, h2r_km, h2p, hp_im,
                   h2p_km, h2z, hz_jm, hz_im, v2, v_im, er2, ep2, ez2, u2);
            store_out(pto(a.oHr + c0m, o), h2r, nt);
            store_out(pto(a.oHp + c0m, o), h2p, nt);
            store_out(pto(a.oHz + c0m, o), h2z, nt);
            store_out(pto(a.oEr + c0m, o), er2, nt);
            store_out(pto(a.oEp + c0m, o), ep2, nt);
            store_out(pto(a.oEz + c0m, o), ez2, nt);
            if (a.dft_plane && km == a.k_mon) {
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw0 = a.twiddle[(size_t)n * a.K + f], tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                    float2 *q0 = pto(a.dft_plane + (size_t)f * 2 * plane + rowc, o);
                    float2 *q1 = pto(a.dft_plane + (size_t)f * 2 * plane + plane + rowc, o);
                    *q0 = c_fma(c_fma(*q0, tw0, e1r_p), tw1, er2);
                    *q1 = c_fma(c_fma(*q1, tw0, e1p_p), tw1, ep2);
                }
            }
            if (a.dft_vol && km >= a.k0 && km < a.k1) {
                const size_t vs = (size_t)nd * plane;
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw0 = a.twiddle[(size_t)n * a.K + f], tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                    float2 *base = a.dft_vol + (size_t)f * 3 * vs + (size_t)(km - a.k0) * plane + rowc;
                    float2 *q0 = pto(base, o), *q1 = pto(base + vs, o), *q2 = pto(base + 2 * vs, o);
                    *q0 = c_fma(c_fma(*q0, tw0, e1r_p), tw1, er2);
                    *q1 = c_fma(c_fma(*q1, tw0, e1p_p), tw1, ep2);
                    *q2 = c_fma(c_fma(*q2, tw0, e1z_p), tw1, ez2);
                }
            }
        }
        er0 = er_kp;
        ep0 = ep_kp;
        h1r_p = h1r;
        h1p_p = h1p;
        h1z_p = h1z;
        e1r_p = e1r;
        e1p_p = e1p;
        e1z_p = e1z;
        u1_p = u1;
        ce_p = ce;
        h2r_km = h2r;
        h2p_km = h2p;
        if constexpr (CARRY) car_p = car_c;
    }
}

// The value a float2 holds in lane l - 1 (shr) or l + 1 (shl) of the wave,
// moved by DPP wave shifts (lane 0, resp. 63, gets zero).  Every lane of the
// wave must execute it.
__device__ __forceinline__ float dpp_f(float x, int ctrl_shl)
{
    const int v = __float_as_int(x);
    return __int_as_float(ctrl_shl ? __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true)
                                   : __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float2 from_lane_below(float2 x) { return make_float2(dpp_f(x.x, 0), dpp_f(x.y, 0)); }
__device__ __forceinline__ float2 from_lane_above(float2 x) { return make_float2(dpp_f(x.x, 1), dpp_f(x.y, 1)); }

// Three whole leap-frog steps (n, n + 1, n + 2) per launch: the two-step
// schedule above one step deeper.  The launch reads level n from one buffer
// set and writes level n + 3 to the other, so each cell's six fields cross
// HBM once per three steps.  Block = (TR + 5) wavefronts x 64 lanes marching
// a z-chunk: wave w on row i0 - 3 + w, lane l on phi cell j0 - 3 + l (j0 =
// three_step_cols(LAY) x tile column), modulo nphi as before.  Step s + 1
// lags step s by one plane; per plane the H half-steps of the three steps
// hand their -r neighbours to the E half-steps through LDS, the E half-steps
// of steps one and two hand their +r neighbours to the next H half-step
// through LDS (double-buffered, the H half-step reads the plane below), and
// the +-phi neighbours move between lanes by DPP shifts.  Exact cells: step
// one H everywhere, E on lanes >= 1 and waves >= 1; step two H on lanes
// 1..62, waves 1..nrow + 3, E on lanes 2..62, waves 2..nrow + 3; step three
// H on lanes 2..61, waves 2..nrow + 2, E (owners) on lanes 3..3 + COLS - 1,
// waves 3..nrow + 2.  A chunk starts three planes early; step one runs two
// planes past its end.  Layer auxiliaries: level n + 1 goes to the
// intermediate set m, level n + 2 to the second intermediate set m2 (written
// only by exact cells, so every block that writes one writes the same
// value), level n + 3 (owners) to the other set.
template <int TR, int LAY>
__device__ __forceinline__ void eh3_body(const StepArgs &a, int n, uint4 tile)
{
    constexpr bool PR = (LAY & 1) != 0, PZ = (LAY & 2) != 0;
    constexpr bool LAYERS = PR || PZ;
    constexpr int NW = TR + 5;
    constexpr int NV = PR ? NW : 1;
    __shared__ float2 s1z[NW][64], s1p[NW][64], s1v[NV][64];
    __shared__ float2 sE1z[2][NW][64], sE1p[2][NW][64], sU1[2][NV][64];
    __shared__ float2 s2z[NW][64], s2p[NW][64], s2v[NV][64];
    __shared__ float2 sE2z[2][NW][64], sE2p[2][NW][64], sU2[2][NV][64];
    __shared__ float2 s3z[NW][64], s3p[NW][64], s3v[NV][64];
    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    const int bx = (int)tile.x, i0 = (int)(tile.y & 0xffffu), nrow = (int)(tile.y >> 16);
    const int kb = (int)(tile.z & 0xffffu), ke = (int)(tile.z >> 16);
    const int i = i0 + w - 3;
    const bool active = w <= nrow + 4;                      // waves above the top halo row idle
    const bool row_ok = active && i >= 0 && i < nr;
    constexpr int COLS = three_step_cols(LAY);
    const int jj = bx * COLS - 3 + lane;
    const int pc = (jj % nphi + nphi) % nphi;               // physical column
    const bool cross_m = pc == 0;                           // lane - 1 holds column nphi - 1
    const bool cross_p = pc == nphi - 1;                    // lane + 1 holds column 0
    const bool own = lane >= 3 && lane < 3 + COLS && jj < nphi && w >= 3 && w <= nrow + 2 && row_ok;
    const int k_lo = max(kb - 3, 0);
    const bool nt = a.nt_stores;
    const int ir = (PR && row_ok) ? slab_row(i, nr, a.pr0, a.pr1) : -1;
    const int ir1 = (PR && row_ok && i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoef rc = a.rows[row_ok ? i : 0];
    const int ic = min(max(i, 0), nr - 1);
    const unsigned o = (unsigned)pc * 8u;
    const unsigned ojp = cross_p ? 0u : o + 8u;
    const unsigned oc = (unsigned)pc * 4u;
    const size_t rowc = (size_t)ic * nphi;
    const bool ip_ok = ic + 1 < nr;
    const size_t dip = ip_ok ? (size_t)nphi : 0;
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const int nd = a.k1 - a.k0;
    // exact lanes of the E and H half-steps of steps one to three (all lanes
    // without layer recursions: inexact cells then only feed inexact cells)
    const bool l_e1 = !LAYERS || lane >= 1, l_h2 = !LAYERS || (lane >= 1 && lane <= 62);
    const bool l_e2 = !LAYERS || (lane >= 2 && lane <= 62), l_h3 = !LAYERS || (lane >= 2 && lane <= 61);

    // carried along z (level: plane): E^n (k); H, E, U, dt/eps of step one
    // (k - 1) and E of step one at k - 2 (DFT); H, E, U of step two (k - 2);
    // H of step three (k - 3)
    float2 er0 = ldo(a.Er + (size_t)k_lo * plane + rowc, o);
    float2 ep0 = ldo(a.Ep + (size_t)k_lo * plane + rowc, o);
    float2 h1r_p = zero2(), h1p_p = zero2(), h1z_p = zero2();
    float2 e1r_p = zero2(), e1p_p = zero2(), e1z_p = zero2(), u1_p = zero2();
    float2 e1r_pp = zero2(), e1p_pp = zero2(), e1z_pp = zero2();
    float2 h2r_p = zero2(), h2p_p = zero2(), h2z_p = zero2();
    float2 e2r_p = zero2(), e2p_p = zero2(), e2z_p = zero2(), u2_p = zero2();
    float2 h3r_km = zero2(), h3p_km = zero2();
    float ce_p = 0.f, ce_pp = 0.f;
    for (int k = k_lo; k <= ke + 1; ++k) {
        const int km = k - 1, km2 = k - 2;
        const PlaneIn in = load_plane(a, min(k, nz - 1), plane, rowc, dip, o, ojp, oc);
        float2 h1r = zero2(), h1p = zero2(), h1z = zero2(), v1 = zero2();
        float2 e1r = zero2(), e1p = zero2(), e1z = zero2(), u1 = zero2();
        float2 er_kp = zero2(), ep_kp = zero2();
        float ce = 0.f;
        const bool step1 = k < nz;
        // ---- step one, H at plane k
        int kz = -1;
        ZCoef zc = {};
        AuxRows x1 = {};
        float2 ez0 = zero2();
        if (step1 && active) {
            kz = PZ ? slab_row(k, nz, a.pz0, a.pz1) : -1;
            if (kz >= 0) zc = a.zrows[k];
            const size_t sr0 = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi : 0;
            const size_t sz0 = kz >= 0 ? ((size_t)kz * nr + ic) * nphi : 0;
            x1 = AuxRows{a.auxR + sr0, a.auxZ + sz0, a.mauxR + sr0, a.mauxZ + sz0};
            const bool kp_ok = k + 1 < nz;
            ez0 = in.ez;
            er_kp = in.er_kp;
            ep_kp = in.ep_kp;
            float2 ez_jp = in.ez_jp, er_jp = in.er_jp;
            float2 ez_ip = in.ez_ip, ep_ip = in.ep_ip;
            h1r = in.hr;
            h1p = in.hp;
            h1z = in.hz;
            ce = in.ce;
            if (!kp_ok) { er_kp = zero2(); ep_kp = zero2(); }
            if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
            if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
            float2 u0 = zero2(), uu1 = zero2();
            if (ir >= 0 && k > 0) {
                u0 = ldo(a.auxR + sr0 + AUX_U_EP * slabR, o);
                if (ir1 >= 0) uu1 = ldo(a.auxR + AUX_U_EP * slabR + ((size_t)k * a.dR + ir1) * nphi, o);
            }
            h_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, row_ok, ez0, er0, ep0, ez_jp, er_jp, er_kp, ep_kp,
                   ez_ip, ep_ip, u0, uu1, h1r, h1p, h1z, v1);
            s1z[w][lane] = h1z;
            s1p[w][lane] = h1p;
            if (PR) s1v[w][lane] = v1;
        }
        __syncthreads();
        // ---- step one, E at plane k
        {
            float2 hz_jm = from_lane_below(h1z), hr_jm = from_lane_below(h1r);
            if (step1 && (k != k_lo || k == 0) && w >= 1 && row_ok) {
                if (l_e1) {
                    if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
                    const float2 hz_im = s1z[w - 1][lane], hp_im = s1p[w - 1][lane];
                    const float2 v_im = PR ? s1v[PR ? w - 1 : 0][lane] : zero2();
                    float2 jr = zero2(), jph = zero2();
                    if (k == a.k_src) sheet_current(a, n, plane, rowc, o, jr, jph);
                    e1r = er0;
                    e1p = ep0;
                    e1z = ez0;
                    e_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, ce, jr, jph, h1r, hr_jm, h1r_p, h1p, hp_im,
                           h1p_p, h1z, hz_jm, hz_im, v1, v_im, e1r, e1p, e1z, u1);
                }
                sE1z[k & 1][w][lane] = e1z;
                sE1p[k & 1][w][lane] = e1p;
                if (PR) sU1[k & 1][PR ? w : 0][lane] = u1;
            }
        }
        // ---- step two, H at plane km
        float2 h2r = zero2(), h2p = zero2(), h2z = zero2(), v2 = zero2();
        const int kz2 = (PZ && km >= 0 && km < nz) ? slab_row(km, nz, a.pz0, a.pz1) : -1;
        ZCoef zc2 = {};
        if (kz2 >= 0) zc2 = a.zrows[km];
        const size_t sr2 = ir >= 0 ? ((size_t)min(max(km, 0), nz - 1) * a.dR + ir) * nphi : 0;
        const size_t sz2 = kz2 >= 0 ? ((size_t)kz2 * nr + ic) * nphi : 0;
        const AuxRows x2 = {a.mauxR + sr2, a.mauxZ + sz2, a.m2auxR + sr2, a.m2auxZ + sz2};
        {
            float2 ez_jp = from_lane_above(e1z_p), er_jp = from_lane_above(e1r_p);
            if (km >= 0 && km < nz && (km > k_lo || k_lo == 0) && w >= 1 && w <= nrow + 3 && row_ok && l_h2) {
                const int b = km & 1;
                if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
                float2 ez_ip = sE1z[b][w + 1][lane], ep_ip = sE1p[b][w + 1][lane];
                if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
                float2 uu1 = zero2();
                if (PR && ir1 >= 0) uu1 = sU1[b][PR ? w + 1 : 0][lane];
                h2r = h1r_p;
                h2p = h1p_p;
                h2z = h1z_p;
                // E of step one at km + 1 is the plane just finished (zero above the top)
                h_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, true, e1z_p, e1r_p, e1p_p, ez_jp, er_jp, e1r,
                       e1p, ez_ip, ep_ip, (ir >= 0 && km > 0) ? u1_p : zero2(), uu1, h2r, h2p, h2z, v2);
            }
        }
        s2z[w][lane] = h2z;
        s2p[w][lane] = h2p;
        if (PR) s2v[w][lane] = v2;
        __syncthreads();
        // ---- step two, E at plane km
        float2 e2r = zero2(), e2p = zero2(), e2z = zero2(), u2 = zero2();
        {
            float2 hz_jm = from_lane_below(h2z), hr_jm = from_lane_below(h2r);
            if (km >= 0 && km < nz && (km > k_lo + 1 || k_lo == 0) && w >= 2 && w <= nrow + 3 && row_ok) {
                if (l_e2) {
                    if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
                    const float2 hz_im = s2z[w - 1][lane], hp_im = s2p[w - 1][lane];
                    const float2 v_im = PR ? s2v[PR ? w - 1 : 0][lane] : zero2();
                    float2 jr = zero2(), jph = zero2();
                    if (km == a.k_src) sheet_current(a, n + 1, plane, rowc, o, jr, jph);
                    e2r = e1r_p;
                    e2p = e1p_p;
                    e2z = e1z_p;
                    e_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, ce_p, jr, jph, h2r, hr_jm, h2r_p, h2p,
                           hp_im, h2p_p, h2z, hz_jm, hz_im, v2, v_im, e2r, e2p, e2z, u2);
                }
                sE2z[km & 1][w][lane] = e2z;
                sE2p[km & 1][w][lane] = e2p;
                if (PR) sU2[km & 1][PR ? w : 0][lane] = u2;
            }
        }
        // ---- step three, H at plane km2
        float2 h3r = zero2(), h3p = zero2(), h3z = zero2(), v3 = zero2();
        const int kz3 = (PZ && km2 >= 0) ? slab_row(km2, nz, a.pz0, a.pz1) : -1;
        ZCoef zc3 = {};
        if (kz3 >= 0) zc3 = a.zrows[km2];
        const size_t c0m = (size_t)max(km2, 0) * plane + rowc;
        const size_t sr3 = ir >= 0 ? ((size_t)max(km2, 0) * a.dR + ir) * nphi : 0;
        const size_t sz3 = kz3 >= 0 ? ((size_t)kz3 * nr + ic) * nphi : 0;
        const AuxRows x3 = {a.m2auxR + sr3, a.m2auxZ + sz3, a.oauxR + sr3, a.oauxZ + sz3};
        const bool store = own && km2 >= kb && km2 < ke;
        {
            float2 ez_jp = from_lane_above(e2z_p), er_jp = from_lane_above(e2r_p);
            if (km2 >= 0 && (km2 > k_lo + 1 || k_lo == 0) && w >= 2 && w <= nrow + 2 && row_ok && l_h3) {
                const int b = km2 & 1;
                if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
                float2 ez_ip = sE2z[b][w + 1][lane], ep_ip = sE2p[b][w + 1][lane];
                if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
                float2 uu1 = zero2();
                if (PR && ir1 >= 0) uu1 = sU2[b][PR ? w + 1 : 0][lane];
                h3r = h2r_p;
                h3p = h2p_p;
                h3z = h2z_p;
                // E of step two at km2 + 1 is the plane step two just finished
                h_cell(a, rc, zc3, i, km2, ir, kz3, slabR, slabZ, x3, o, store, e2z_p, e2r_p, e2p_p, ez_jp, er_jp,
                       e2r, e2p, ez_ip, ep_ip, (ir >= 0 && km2 > 0) ? u2_p : zero2(), uu1, h3r, h3p, h3z, v3);
            }
        }
        s3z[w][lane] = h3z;
        s3p[w][lane] = h3p;
        if (PR) s3v[w][lane] = v3;
        __syncthreads();
        // ---- step three, E at plane km2 (owners), stores and DFT
        {
            float2 hz_jm = from_lane_below(h3z), hr_jm = from_lane_below(h3r);
            if (store) {
                if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
                const float2 hz_im = s3z[w - 1][lane], hp_im = s3p[w - 1][lane];
                const float2 v_im = PR ? s3v[PR ? w - 1 : 0][lane] : zero2();
                float2 jr = zero2(), jph = zero2();
                if (km2 == a.k_src) sheet_current(a, n + 2, plane, rowc, o, jr, jph);
                float2 er3 = e2r_p, ep3 = e2p_p, ez3 = e2z_p, u3;
                e_cell(a, rc, zc3, i, km2, ir, kz3, slabR, slabZ, x3, o, ce_pp, jr, jph, h3r, hr_jm, h3r_km, h3p,
                       hp_im, h3p_km, h3z, hz_jm, hz_im, v3, v_im, er3, ep3, ez3, u3);
                store_out(pto(a.oHr + c0m, o), h3r, nt);
                store_out(pto(a.oHp + c0m, o), h3p, nt);
                store_out(pto(a.oHz + c0m, o), h3z, nt);
                store_out(pto(a.oEr + c0m, o), er3, nt);
                store_out(pto(a.oEp + c0m, o), ep3, nt);
                store_out(pto(a.oEz + c0m, o), ez3, nt);
                if (a.dft_plane && km2 == a.k_mon) {
                    for (int f = 0; f < a.K; ++f) {
                        const float2 tw0 = a.twiddle[(size_t)n * a.K + f];
                        const float2 tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                        const float2 tw2 = a.twiddle[(size_t)(n + 2) * a.K + f];
                        float2 *q0 = pto(a.dft_plane + (size_t)f * 2 * plane + rowc, o);
                        float2 *q1 = pto(a.dft_plane + (size_t)f * 2 * plane + plane + rowc, o);
                        *q0 = c_fma(c_fma(c_fma(*q0, tw0, e1r_pp), tw1, e2r_p), tw2, er3);
                        *q1 = c_fma(c_fma(c_fma(*q1, tw0, e1p_pp), tw1, e2p_p), tw2, ep3);
                    }
                }
                if (a.dft_vol && km2 >= a.k0 && km2 < a.k1) {
                    const size_t vs = (size_t)nd * plane;
                    for (int f = 0; f < a.K; ++f) {
                        const float2 tw0 = a.twiddle[(size_t)n * a.K + f];
                        const float2 tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                        const float2 tw2 = a.twiddle[(size_t)(n + 2) * a.K + f];
                        float2 *base = a.dft_vol + (size_t)f * 3 * vs + (size_t)(km2 - a.k0) * plane + rowc;
                        float2 *q0 = pto(base, o), *q1 = pto(base + vs, o), *q2 = pto(base + 2 * vs, o);
                        *q0 = c_fma(c_fma(c_fma(*q0, tw0, e1r_pp), tw1, e2r_p), tw2, er3);
                        *q1 = c_fma(c_fma(c_fma(*q1, tw0, e1p_pp), tw1, e2p_p), tw2, ep3);
                        *q2 = c_fma(c_fma(c_fma(*q2, tw0, e1z_pp), tw1, e2z_p), tw2, ez3);
                    }
                }
            }
        }
        er0 = er_kp;
        ep0 = ep_kp;
        e1r_pp = e1r_p;
        e1p_pp = e1p_p;
        e1z_pp = e1z_p;
        h1r_p = h1r;
        h1p_p = h1p;
        h1z_p = h1z;
        e1r_p = e1r;
        e1p_p = e1p;
        e1z_p = e1z;
        u1_p = u1;
        ce_pp = ce_p;
        ce_p = ce;
        h3r_km = h3r;
        h3p_km = h3p;
        h2r_p = h2r;
        h2p_p = h2p;
        h2z_p = h2z;
        e2r_p = e2r;
        e2p_p = e2p;
        e2z_p = e2z;
        u2_p = u2;
    }
}

// The two-step schedule above with the flat (r, phi) mapping, for narrow
// zones (nphi <= FLAT_TWO_MAX_PHI): a block of FLAT_BLOCK threads holds
// RB = FLAT_BLOCK / nphi whole rows, thread t on row slot s = t / nphi
// (radial row i0 - 2 + s) and phi cell j = t mod nphi, so a block's loads and
// stores cover consecutive cells.  Slots 0, 1 and nrow + 2 are the radial
// halo (nrow <= RB - 3 owned rows); the +-phi neighbours are the adjacent
// threads of the row, across the Bloch seam (with its factor) at j = 0 and
// j = nphi - 1, so every column is exact and owned: no azimuthal halo.  The
// tile's phi block (first word) is 0.
template <int LAY>
__device__ __forceinline__ void eh2_flat_body(const StepArgs &a, int n, uint4 tile)
{
    constexpr bool PR = (LAY & 1) != 0, PZ = (LAY & 2) != 0;
    constexpr int NB = FLAT_BLOCK;
    constexpr int NV = PR ? NB : 1;
    __shared__ float2 s1z[NB], s1r[NB], s1p[NB], s1v[NV];
    __shared__ float2 sEz[2][NB], sEr[2][NB], sEp[2][NB], sU[2][NV];
    __shared__ float2 s2z[NB], s2r[NB], s2p[NB], s2v[NV];
    const int t = threadIdx.x;
    const int nphi = a.nphi, nr = a.nr, nz = a.nz;
    const size_t plane = (size_t)nr * nphi;
    const int i0 = (int)(tile.y & 0xffffu), nrow = (int)(tile.y >> 16);
    const int kb = (int)(tile.z & 0xffffu), ke = (int)(tile.z >> 16);
    const int sl = t / nphi, j = t - sl * nphi;
    const int i = i0 + sl - 2;
    const bool active = sl <= nrow + 2;                     // slots above the top halo row idle
    const bool row_ok = active && i >= 0 && i < nr;
    const bool cross_m = j == 0;                            // -phi neighbour is column nphi - 1
    const bool cross_p = j == nphi - 1;                     // +phi neighbour is column 0
    const bool own = sl >= 2 && sl <= nrow + 1 && row_ok;
    // LDS slots of the neighbours; only active slots read them, and the
    // clamps keep every index inside the arrays whatever the thread
    const int t_jm = min(cross_m ? t + nphi - 1 : t - 1, NB - 1);
    const int t_jp = cross_p ? t - (nphi - 1) : min(t + 1, NB - 1);
    const int t_im = sl >= 1 ? t - nphi : t;
    const int t_ip = min(t + nphi, NB - 1);
    const int k_lo = max(kb - 2, 0);
    const bool nt = a.nt_stores;
    const int ir = (PR && row_ok) ? slab_row(i, nr, a.pr0, a.pr1) : -1;
    const int ir1 = (PR && row_ok && i + 1 < nr) ? slab_row(i + 1, nr, a.pr0, a.pr1) : -1;
    const RowCoef rc = a.rows[row_ok ? i : 0];
    const int ic = min(max(i, 0), nr - 1);
    const unsigned o = (unsigned)j * 8u;
    const unsigned ojp = cross_p ? 0u : o + 8u;
    const unsigned oc = (unsigned)j * 4u;
    const size_t rowc = (size_t)ic * nphi;
    const bool ip_ok = ic + 1 < nr;
    const size_t dip = ip_ok ? (size_t)nphi : 0;
    const size_t slabR = (size_t)nz * a.dR * nphi;
    const size_t slabZ = (size_t)a.dZ * plane;
    const int nd = a.k1 - a.k0;

    // carried along z as in the two-step kernel: E^n at k; H^{n+1/2},
    // E^{n+1}, U^{n+1}, dt/eps at k - 1; H^{n+3/2} at k - 2
    float2 er0 = ldo(a.Er + (size_t)k_lo * plane + rowc, o);
    float2 ep0 = ldo(a.Ep + (size_t)k_lo * plane + rowc, o);
    float2 h1r_p = zero2(), h1p_p = zero2(), h1z_p = zero2();
    float2 e1r_p = zero2(), e1p_p = zero2(), e1z_p = zero2(), u1_p = zero2();
    float2 h2r_km = zero2(), h2p_km = zero2();
    float ce_p = 0.f;
    constexpr bool PF = !PR;
    PlaneIn cur = load_plane(a, k_lo, plane, rowc, dip, o, ojp, oc);
    for (int k = k_lo; k <= ke; ++k) {
        const int km = k - 1;
        PlaneIn in;
        if (!PF) {
            in = load_plane(a, min(k, nz - 1), plane, rowc, dip, o, ojp, oc);
        } else {
            in = cur;
            cur = load_plane(a, min(k + 1, min(ke, nz - 1)), plane, rowc, dip, o, ojp, oc);
        }
        float2 h1r = zero2(), h1p = zero2(), h1z = zero2(), v1 = zero2();
        float2 e1r = zero2(), e1p = zero2(), e1z = zero2(), u1 = zero2();
        float2 er_kp = zero2(), ep_kp = zero2();
        float ce = 0.f;
        const bool step1 = k < nz;
        // ---- step one, H^{n+1/2} at plane k (every active slot)
        int kz = -1;
        ZCoef zc = {};
        AuxRows x1 = {};
        float2 ez0 = zero2();
        if (step1 && active) {
            kz = PZ ? slab_row(k, nz, a.pz0, a.pz1) : -1;
            if (kz >= 0) zc = a.zrows[k];
            const size_t sr0 = ir >= 0 ? ((size_t)k * a.dR + ir) * nphi : 0;
            const size_t sz0 = kz >= 0 ? ((size_t)kz * nr + ic) * nphi : 0;
            x1 = {a.auxR + sr0, a.auxZ + sz0, a.mauxR + sr0, a.mauxZ + sz0};
            const bool kp_ok = k + 1 < nz;
            ez0 = in.ez;
            er_kp = in.er_kp;
            ep_kp = in.ep_kp;
            float2 ez_jp = in.ez_jp, er_jp = in.er_jp;
            float2 ez_ip = in.ez_ip, ep_ip = in.ep_ip;
            h1r = in.hr;
            h1p = in.hp;
            h1z = in.hz;
            ce = in.ce;
            if (!kp_ok) { er_kp = zero2(); ep_kp = zero2(); }
            if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
            if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
            float2 u0 = zero2(), uu1 = zero2();
            if (ir >= 0 && k > 0) {
                u0 = ldo(x1.sR + AUX_U_EP * slabR, o);
                if (ir1 >= 0) uu1 = ldo(a.auxR + AUX_U_EP * slabR + ((size_t)k * a.dR + ir1) * nphi, o);
            }
            h_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, row_ok, ez0, er0, ep0, ez_jp, er_jp, er_kp, ep_kp,
                   ez_ip, ep_ip, u0, uu1, h1r, h1p, h1z, v1);
            s1z[t] = h1z;
            s1r[t] = h1r;
            s1p[t] = h1p;
            if (PR) s1v[PR ? t : 0] = v1;
        }
        __syncthreads();
        // ---- step one, E^{n+1} at plane k (exact on slots >= 1)
        if (step1 && (k != k_lo || k == 0) && sl >= 1 && row_ok) {
            float2 hz_jm = s1z[t_jm], hr_jm = s1r[t_jm];
            if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
            const float2 hz_im = s1z[t_im], hp_im = s1p[t_im];
            const float2 v_im = PR ? s1v[PR ? t_im : 0] : zero2();
            float2 jr = zero2(), jph = zero2();
            if (k == a.k_src) sheet_current(a, n, plane, rowc, o, jr, jph);
            e1r = er0;
            e1p = ep0;
            e1z = ez0;
            e_cell(a, rc, zc, i, k, ir, kz, slabR, slabZ, x1, o, ce, jr, jph, h1r, hr_jm, h1r_p, h1p, hp_im, h1p_p,
                   h1z, hz_jm, hz_im, v1, v_im, e1r, e1p, e1z, u1);
            sEz[k & 1][t] = e1z;
            sEr[k & 1][t] = e1r;
            sEp[k & 1][t] = e1p;
            if (PR) sU[k & 1][PR ? t : 0] = u1;
        }
        // ---- step two, H^{n+3/2} at plane km (exact on slots 1 .. nrow + 1)
        float2 h2r = zero2(), h2p = zero2(), h2z = zero2(), v2 = zero2();
        const bool h2_plane = km >= 0 && (km > k_lo || km == 0);
        const int kz2 = (PZ && km >= 0) ? slab_row(km, nz, a.pz0, a.pz1) : -1;
        ZCoef zc2 = {};
        if (kz2 >= 0) zc2 = a.zrows[km];
        const size_t c0m = (size_t)max(km, 0) * plane + rowc;
        const size_t sr2 = ir >= 0 ? ((size_t)max(km, 0) * a.dR + ir) * nphi : 0;
        const size_t sz2 = kz2 >= 0 ? ((size_t)kz2 * nr + ic) * nphi : 0;
        const AuxRows x2 = {a.mauxR + sr2, a.mauxZ + sz2, a.oauxR + sr2, a.oauxZ + sz2};
        const bool store = own && km >= kb && km < ke;
        if (h2_plane && sl >= 1 && sl <= nrow + 1 && row_ok) {
            const int b = km & 1;
            float2 ez_jp = sEz[b][t_jp], er_jp = sEr[b][t_jp];
            if (cross_p) { ez_jp = c_mul(a.seam_p, ez_jp); er_jp = c_mul(a.seam_p, er_jp); }
            float2 ez_ip = sEz[b][t_ip], ep_ip = sEp[b][t_ip];
            if (!ip_ok) { ez_ip = zero2(); ep_ip = zero2(); }
            float2 uu1 = zero2();
            if (PR && ir1 >= 0) uu1 = sU[b][PR ? t_ip : 0];
            h2r = h1r_p;
            h2p = h1p_p;
            h2z = h1z_p;
            // E^{n+1} at km + 1 is the plane step one just finished (zero above the top)
            h_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, store, e1z_p, e1r_p, e1p_p, ez_jp, er_jp, e1r,
                   e1p, ez_ip, ep_ip, (ir >= 0 && km > 0) ? u1_p : zero2(), uu1, h2r, h2p, h2z, v2);
        }
        s2z[t] = h2z;
        s2r[t] = h2r;
        s2p[t] = h2p;
        if (PR) s2v[PR ? t : 0] = v2;
        __syncthreads();
        // ---- step two, E^{n+2} at plane km (owners), stores and DFT
        if (store) {
            float2 hz_jm = s2z[t_jm], hr_jm = s2r[t_jm];
            if (cross_m) { hz_jm = c_mul(a.seam_m, hz_jm); hr_jm = c_mul(a.seam_m, hr_jm); }
            const float2 hz_im = s2z[t_im], hp_im = s2p[t_im];
            const float2 v_im = PR ? s2v[PR ? t_im : 0] : zero2();
            float2 jr = zero2(), jph = zero2();
            if (km == a.k_src) sheet_current(a, n + 1, plane, rowc, o, jr, jph);
            float2 er2 = e1r_p, ep2 = e1p_p, ez2 = e1z_p, u2;
            e_cell(a, rc, zc2, i, km, ir, kz2, slabR, slabZ, x2, o, ce_p, jr, jph, h2r, hr_jm, h2r_km, h2p, hp_im,
                   h2p_km, h2z, hz_jm, hz_im, v2, v_im, er2, ep2, ez2, u2);
            store_out(pto(a.oHr + c0m, o), h2r, nt);
            store_out(pto(a.oHp + c0m, o), h2p, nt);
            store_out(pto(a.oHz + c0m, o), h2z, nt);
            store_out(pto(a.oEr + c0m, o), er2, nt);
            store_out(pto(a.oEp + c0m, o), ep2, nt);
            store_out(pto(a.oEz + c0m, o), ez2, nt);
            if (a.dft_plane && km == a.k_mon) {
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw0 = a.twiddle[(size_t)n * a.K + f], tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                    float2 *q0 = pto(a.dft_plane + (size_t)f * 2 * plane + rowc, o);
                    float2 *q1 = pto(a.dft_plane + (size_t)f * 2 * plane + plane + rowc, o);
                    *q0 = c_fma(c_fma(*q0, tw0, e1r_p), tw1, er2);
                    *q1 = c_fma(c_fma(*q1, tw0, e1p_p), tw1, ep2);
                }
            }
            if (a.dft_vol && km >= a.k0 && km < a.k1) {
                const size_t vs = (size_t)nd * plane;
                for (int f = 0; f < a.K; ++f) {
                    const float2 tw0 = a.twiddle[(size_t)n * a.K + f], tw1 = a.twiddle[(size_t)(n + 1) * a.K + f];
                    float2 *base = a.dft_vol + (size_t)f * 3 * vs + (size_t)(km - a.k0) * plane + rowc;
                    float2 *q0 = pto(base, o), *q1 = pto(base + vs, o), *q2 = pto(base + 2 * vs, o);
                    *q0 = c_fma(c_fma(*q0, tw0, e1r_p), tw1, er2);
                    *q1 = c_fma(c_fma(*q1, tw0, e1p_p), tw1, ep2);
                    *q2 = c_fma(c_fma(*q2, tw0, e1z_p), tw1, ez2);
                }
            }
        }
        er0 = er_kp;
        ep0 = ep_kp;
        h1r_p = h1r;
        h1p_p = h1p;
        h1z_p = h1z;
        e1r_p = e1r;
        e1p_p = e1p;
        e1z_p = e1z;
        u1_p = u1;
        ce_p = ce;
        h2r_km = h2r;
        h2p_km = h2p;
    }
}

// Workgroups are dealt round-robin to the 8 XCDs; renumbering them so that
// each XCD gets one contiguous range of tiles keeps the halo rows, columns and
// chunk prologue planes that neighbouring tiles share in the same L2.
__device__ __forceinline__ unsigned xcd_order(unsigned p, unsigned nblk, int on)
{
    if (!on || nblk < 8) return p;
    const unsigned per = nblk / 8, rem = nblk % 8, x = p % 8, s = p / 8;
    return x * per + min(x, rem) + s;
}

template <int BY>
__global__ __launch_bounds__(BX * BY) void h_step_kernel(StepArgs a, int n)
{
    h_step_body<BY>(a, n, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int BY>
__global__ __launch_bounds__(BX * BY) void e_step_kernel(StepArgs a, int n)
{
    e_step_body<BY>(a, n, blockIdx.x, blockIdx.y, blockIdx.z);
}

// FP64 instantiation of the in-place pair (verification runs)
template <int BY>
__global__ __launch_bounds__(BX * BY) void h_step_kernel64(StepArgs64 a, int n)
{
    h_step_body<BY, false, double>(a, n, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int BY>
__global__ __launch_bounds__(BX * BY) void e_step_kernel64(StepArgs64 a, int n)
{
    e_step_body<BY, false, double>(a, n, blockIdx.x, blockIdx.y, blockIdx.z);
}

__global__ __launch_bounds__(FLAT_BLOCK) void h_step_flat(StepArgs a, int n)
{
    h_step_body<1, true>(a, n, blockIdx.x, 0, blockIdx.z);
}

__global__ __launch_bounds__(FLAT_BLOCK) void e_step_flat(StepArgs a, int n)
{
    e_step_body<1, true>(a, n, blockIdx.x, 0, blockIdx.z);
}

__global__ __launch_bounds__(FLAT_BLOCK) void eh_flat_kernel(StepArgs a, int n)
{
    eh_flat_body(a, n, blockIdx.x, blockIdx.y);
}

template <int TR>
__global__ __launch_bounds__(64 * (TR + 1)) void eh_fused_kernel(StepArgs a, int n)
{
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned nblk = gx * gy * gridDim.z;
    const unsigned p = xcd_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), nblk, a.xcd_remap);
    eh_fused_body<TR>(a, n, p, gx, gy);
}

template <int TR, int LAY>
__global__ __launch_bounds__(64 * (TR + 5)) void eh3_kernel(StepArgs a, int n)
{
    eh3_body<TR, LAY>(a, n, a.tiles[blockIdx.x]);
}

template <int TR, int LAY, bool CARRY = false>
__global__ __launch_bounds__(64 * (TR + 3)) void eh2_kernel(StepArgs a, int n)
{
    eh2_body<TR, LAY, CARRY>(a, n, a.tiles[blockIdx.x]);
}

template <int LAY>
__global__ __launch_bounds__(FLAT_BLOCK) void eh2_flat_kernel(StepArgs a, int n)
{
    eh2_flat_body<LAY>(a, n, a.tiles[blockIdx.x]);
}

// Batched launches: one 1-D grid covers the tiles of many zones of uneven
// size; block b belongs to the zone whose prefix range holds it.

// A pointer held in device memory that addresses global memory, read as a
// global-address-space pointer: the compiler then issues global (not flat)
// loads and stores through it, whose completion the LDS waits do not include.
template <class T>
__device__ __forceinline__ T *load_global_ptr(T *const *slot)
{
    using G = __attribute__((address_space(1))) T *;
    return (T *)(*static_cast<const G *>(static_cast<const void *>(slot)));
}

// A zone's arguments from the batch table, every pointer read as global.
__device__ __forceinline__ StepArgs zone_args(const StepArgs *tab, int zi)
{
    const StepArgs *e = tab + zi;
    StepArgs a = *e;
    a.Er = load_global_ptr(&e->Er); a.Ep = load_global_ptr(&e->Ep); a.Ez = load_global_ptr(&e->Ez);
    a.Hr = load_global_ptr(&e->Hr); a.Hp = load_global_ptr(&e->Hp); a.Hz = load_global_ptr(&e->Hz);
    a.oEr = load_global_ptr(&e->oEr); a.oEp = load_global_ptr(&e->oEp); a.oEz = load_global_ptr(&e->oEz);
    a.oHr = load_global_ptr(&e->oHr); a.oHp = load_global_ptr(&e->oHp); a.oHz = load_global_ptr(&e->oHz);
    a.ceps = load_global_ptr(&e->ceps);
    a.auxR = load_global_ptr(&e->auxR); a.auxZ = load_global_ptr(&e->auxZ);
    a.oauxR = load_global_ptr(&e->oauxR); a.oauxZ = load_global_ptr(&e->oauxZ);
    a.mauxR = load_global_ptr(&e->mauxR); a.mauxZ = load_global_ptr(&e->mauxZ);
    a.rows = load_global_ptr(&e->rows); a.zrows = load_global_ptr(&e->zrows);
    a.pattern = load_global_ptr(&e->pattern); a.profile = load_global_ptr(&e->profile);
    a.twiddle = load_global_ptr(&e->twiddle);
    a.dft_plane = load_global_ptr(&e->dft_plane); a.dft_vol = load_global_ptr(&e->dft_vol);
    a.tiles = load_global_ptr(&e->tiles);
    return a;
}
__device__ __forceinline__ int batch_zone(const unsigned *prefix, int nzones, unsigned b)
{
    int lo = 0, hi = nzones - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int BY>
__global__ __launch_bounds__(BX * BY) void h_step_batch(BatchArgs b, int n_rel)
{
    const int zi = batch_zone(b.prefix, b.nzones, blockIdx.x);
    const StepArgs a = zone_args(b.tab, zi);
    const unsigned local = blockIdx.x - b.prefix[zi];
    const unsigned gx = (a.nphi + BX - 1) / BX, gy = (a.nr + BY - 1) / BY;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    h_step_body<BY>(a, n, local % gx, (local / gx) % gy, local / (gx * gy));
}

template <int BY>
__global__ __launch_bounds__(BX * BY) void e_step_batch(BatchArgs b, int n_rel)
{
    const int zi = batch_zone(b.prefix, b.nzones, blockIdx.x);
    const StepArgs a = zone_args(b.tab, zi);
    const unsigned local = blockIdx.x - b.prefix[zi];
    const unsigned gx = (a.nphi + BX - 1) / BX, gy = (a.nr + BY - 1) / BY;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    e_step_body<BY>(a, n, local % gx, (local / gx) % gy, local / (gx * gy));
}

__global__ __launch_bounds__(FLAT_BLOCK) void h_flat_batch(BatchArgs b, int n_rel)
{
    const int zi = batch_zone(b.prefix, b.nzones, blockIdx.x);
    const StepArgs a = zone_args(b.tab, zi);
    const unsigned local = blockIdx.x - b.prefix[zi];
    const unsigned gq = ((unsigned)a.nr * (unsigned)a.nphi + FLAT_BLOCK - 1) / FLAT_BLOCK;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    h_step_body<1, true>(a, n, local % gq, 0, local / gq);
}

__global__ __launch_bounds__(FLAT_BLOCK) void e_flat_batch(BatchArgs b, int n_rel)
{
    const int zi = batch_zone(b.prefix, b.nzones, blockIdx.x);
    const StepArgs a = zone_args(b.tab, zi);
    const unsigned local = blockIdx.x - b.prefix[zi];
    const unsigned gq = ((unsigned)a.nr * (unsigned)a.nphi + FLAT_BLOCK - 1) / FLAT_BLOCK;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    e_step_body<1, true>(a, n, local % gq, 0, local / gq);
}

template <int TR>
__global__ __launch_bounds__(64 * (TR + 1)) void eh_fused_batch(BatchArgs b, int n_rel)
{
    const unsigned g = xcd_order(blockIdx.x, gridDim.x, b.xcd_remap);
    const int zi = batch_zone(b.prefix, b.nzones, g);
    // plain table read: with global pointers this kernel measured 6-11 % slower
    const StepArgs a = b.tab[zi];
    const unsigned gx = (a.nphi + FUSED_COLS - 1) / FUSED_COLS, gy = (a.nr + TR - 1) / TR;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    eh_fused_body<TR>(a, n, g - b.prefix[zi], gx, gy);
}

__global__ __launch_bounds__(FLAT_BLOCK) void eh_flat_batch(BatchArgs b, int n_rel)
{
    const int zi = batch_zone(b.prefix, b.nzones, blockIdx.x);
    const StepArgs a = zone_args(b.tab, zi);
    const unsigned local = blockIdx.x - b.prefix[zi];
    const unsigned R = FLAT_BLOCK / a.nphi - 1;
    const unsigned gq = ((unsigned)a.nr + R - 1) / R;
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    eh_flat_body(a, n, local % gq, local / gq);
}

template <int TR, int LAY, bool CARRY = false>
__global__ __launch_bounds__(64 * (TR + 3)) void eh2_batch(BatchArgs b, int n_rel)
{
    const uint4 tile = b.tiles[blockIdx.x];
    const StepArgs a = zone_args(b.tab, (int)tile.w);
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    eh2_body<TR, LAY, CARRY>(a, n, tile);
}

template <int LAY>
__global__ __launch_bounds__(FLAT_BLOCK) void eh2_flat_batch(BatchArgs b, int n_rel)
{
    const uint4 tile = b.tiles[blockIdx.x];
    const StepArgs a = zone_args(b.tab, (int)tile.w);
    const int n = n_rel + (b.n_base ? *b.n_base : 0);
    eh2_flat_body<LAY>(a, n, tile);
}

__global__ void advance_step_kernel(int *n_base, int by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_base += by;
}

__global__ void set_int_kernel(int *p, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void fill_kernel(float2 *p, size_t n)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; q < n; q += stride) p[q] = zero2();
}

__global__ void fill64_kernel(double2 *p, size_t n)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; q < n; q += stride) p[q] = make_double2(0.0, 0.0);
}

__global__ void inv_eps64_kernel(double *ceps, const double *eps, size_t n, double dt)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) ceps[q] = dt / eps[q];
}

__global__ void inv_eps_kernel(float *ceps, const float *eps, size_t n, double dt)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) ceps[q] = (float)(dt / (eps ? (double)eps[q] : 1.0));
}

// eq. (6): eps = eps_bg + rho (eps_hi - eps_bg), rounded to FP32, then dt/eps
__global__ void design_kernel(float *ceps, const float *rho, size_t n, double eps_bg, double eps_hi, double dt)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) {
        float e = (float)(eps_bg + (double)rho[q] * (eps_hi - eps_bg));
        ceps[q] = (float)(dt / (double)e);
    }
}

__global__ void seed_u_kernel(float2 *U, const float2 *Ep, int nr, int nphi, int nz, int pr0, int pr1, float dt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int k = blockIdx.z;
    if (j >= nphi) return;
    const int ir = slab_row(i, nr, pr0, pr1);
    if (ir < 0) return;
    const int dR = pr0 + pr1;
    float2 e = Ep[((size_t)k * nr + i) * nphi + j];
    U[((size_t)k * dR + ir) * nphi + j] = make_float2(dt * e.x, dt * e.y);
}

__global__ void adjoint_pattern_kernel(float2 *pat, const float2 *g, const float2 *fac, int K, int nr, int nphi)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int ka = blockIdx.z;            // frequency * 2 + component
    if (j >= nphi) return;
    const size_t q = ((size_t)ka * nr + i) * nphi + j;
    pat[q] = c_mul(g[q], fac[(size_t)ka * nr + i]);
}

// grad = scale * sum_k sum_a Re[wr(k,a,i) wz(k,a,kd) X E]; fixed summation order
__global__ void overlap_kernel(float *grad, const float2 *fwd, const float2 *adj, const float2 *wr,
                               const float2 *wz, int K, int nd, int nr, int nphi, float scale)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int kd = blockIdx.z;
    if (j >= nphi) return;
    const size_t plane = (size_t)nr * nphi;
    const size_t vs = (size_t)nd * plane;
    const size_t off = (size_t)kd * plane + (size_t)i * nphi + j;
    float acc = 0.f;
    for (int f = 0; f < K; ++f)
        for (int a = 0; a < 3; ++a) {
            const size_t q = ((size_t)f * 3 + a) * vs + off;
            const float2 w = c_mul(wr[((size_t)f * 3 + a) * nr + i], wz[((size_t)f * 3 + a) * nd + kd]);
            const float2 p = c_mul(adj[q], fwd[q]);
            acc += w.x * p.x - w.y * p.y;
        }
    grad[off] = scale * acc;
}

__global__ void nonfinite_kernel(const float2 *p, size_t n, int *flag)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; q < n; q += stride) {
        float2 v = p[q];
        if (!isfinite(v.x) || !isfinite(v.y)) *flag = 1;
    }
}

// every thread scans a grid-strided share of each array; the first sample out
// of bounds (a NaN fails the comparison) raises the flag and ends the thread
__global__ void watch_kernel(WatchArgs w)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int c = 0; c < 6; ++c) {
        const float2 *p = w.f[c];
        if (!p) continue;
        for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < w.n; q += stride) {
            const float2 v = p[q];
            if (!(v.x * v.x + v.y * v.y < w.bound2)) {
                *w.flag = 1;
                return;
            }
        }
    }
}

}  // namespace

template <int BY>
void launch_pair(const StepArgs &a, int n, hipStream_t s, bool h)
{
    dim3 block(BX, BY, 1);
    dim3 grid((a.nphi + BX - 1) / BX, (a.nr + BY - 1) / BY, (a.nz + a.kchunk - 1) / a.kchunk);
    if (h) hipLaunchKernelGGL(h_step_kernel<BY>, grid, block, 0, s, a, n);
    else hipLaunchKernelGGL(e_step_kernel<BY>, grid, block, 0, s, a, n);
}

void launch_step(const StepArgs &a, int n, hipStream_t s, bool h)
{
    if (a.tile_rows == FLAT_ROWS) {
        dim3 grid(((unsigned)a.nr * (unsigned)a.nphi + FLAT_BLOCK - 1) / FLAT_BLOCK, 1,
                  (a.nz + a.kchunk - 1) / a.kchunk);
        if (h) hipLaunchKernelGGL(h_step_flat, grid, dim3(FLAT_BLOCK), 0, s, a, n);
        else hipLaunchKernelGGL(e_step_flat, grid, dim3(FLAT_BLOCK), 0, s, a, n);
        return;
    }
    switch (a.tile_rows) {
    case 1: launch_pair<1>(a, n, s, h); break;
    case 2: launch_pair<2>(a, n, s, h); break;
    case 8: launch_pair<8>(a, n, s, h); break;
    case 16: launch_pair<16>(a, n, s, h); break;
    default: launch_pair<4>(a, n, s, h); break;
    }
}

void launch_h_step(const StepArgs &a, int n, hipStream_t s) { launch_step(a, n, s, true); }

namespace {
constexpr int BY64 = 4;
dim3 grid64(const StepArgs64 &a)
{
    return dim3((a.nphi + BX - 1) / BX, (a.nr + BY64 - 1) / BY64, (a.nz + a.kchunk - 1) / a.kchunk);
}
}  // namespace

void launch_h_step64(const StepArgs64 &a, int n, hipStream_t s)
{
    hipLaunchKernelGGL(h_step_kernel64<BY64>, grid64(a), dim3(BX, BY64, 1), 0, s, a, n);
}

void launch_e_step64(const StepArgs64 &a, int n, hipStream_t s)
{
    hipLaunchKernelGGL(e_step_kernel64<BY64>, grid64(a), dim3(BX, BY64, 1), 0, s, a, n);
}

template <int TR>
void launch_fused_tr(const StepArgs &a, int n, hipStream_t s)
{
    dim3 block(64, TR + 1, 1);
    dim3 grid((a.nphi + FUSED_COLS - 1) / FUSED_COLS, (a.nr + TR - 1) / TR, (a.nz + a.kchunk - 1) / a.kchunk);
    hipLaunchKernelGGL(eh_fused_kernel<TR>, grid, block, 0, s, a, n);
}

void launch_fused_step(const StepArgs &a, int n, hipStream_t s)
{
    if (a.tile_rows == FLAT_FUSED_ROWS) {
        const unsigned R = FLAT_BLOCK / a.nphi - 1;
        dim3 grid(((unsigned)a.nr + R - 1) / R, (a.nz + a.kchunk - 1) / a.kchunk, 1);
        hipLaunchKernelGGL(eh_flat_kernel, grid, dim3(FLAT_BLOCK), 0, s, a, n);
        return;
    }
    switch (a.tile_rows) {
    case 3: launch_fused_tr<3>(a, n, s); break;
    case 15: launch_fused_tr<15>(a, n, s); break;
    default: launch_fused_tr<7>(a, n, s); break;
    }
}

void launch_e_step(const StepArgs &a, int n, hipStream_t s) { launch_step(a, n, s, false); }

template <int TR>
void launch_batch_two_tr(const BatchArgs &b, unsigned ntiles, int lay, int n_rel, hipStream_t s)
{
    dim3 block(64, TR + 3, 1);
    if (lay == 0) hipLaunchKernelGGL((eh2_batch<TR, 0>), dim3(ntiles), block, 0, s, b, n_rel);
    else if (lay == 2) hipLaunchKernelGGL((eh2_batch<TR, 2, true>), dim3(ntiles), block, 0, s, b, n_rel);
    else hipLaunchKernelGGL((eh2_batch<TR, 3>), dim3(ntiles), block, 0, s, b, n_rel);
}

void launch_batch_two(const BatchArgs &b, unsigned ntiles, int tile_rows, int lay, int n_rel, hipStream_t s)
{
    if (ntiles == 0) return;
    if (tile_rows == FLAT_TWO_ROWS) {
        if (lay == 0) hipLaunchKernelGGL(eh2_flat_batch<0>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, b, n_rel);
        else if (lay == 2) hipLaunchKernelGGL(eh2_flat_batch<2>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, b, n_rel);
        else hipLaunchKernelGGL(eh2_flat_batch<3>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, b, n_rel);
    } else if (lay == 1) {
        hipLaunchKernelGGL((eh2_batch<TWO_CARRY_ROWS, 3, true>), dim3(ntiles), dim3(64, TWO_CARRY_ROWS + 3, 1), 0, s,
                           b, n_rel);
    } else if (lay == 4) {
        hipLaunchKernelGGL((eh2_batch<TWO_RBAND_ROWS, 1, true>), dim3(ntiles), dim3(64, TWO_RBAND_ROWS + 3, 1), 0, s,
                           b, n_rel);
    } else if (tile_rows == 13) launch_batch_two_tr<13>(b, ntiles, lay, n_rel, s);
    else launch_batch_two_tr<5>(b, ntiles, lay, n_rel, s);
}

template <int TR>
void launch_two_tr(const StepArgs &a, int n, unsigned ntiles, int lay, hipStream_t s)
{
    dim3 block(64, TR + 3, 1);
    if (lay == 0) hipLaunchKernelGGL((eh2_kernel<TR, 0>), dim3(ntiles), block, 0, s, a, n);
    else if (lay == 2) hipLaunchKernelGGL((eh2_kernel<TR, 2, true>), dim3(ntiles), block, 0, s, a, n);
    else hipLaunchKernelGGL((eh2_kernel<TR, 3>), dim3(ntiles), block, 0, s, a, n);
}

void launch_two_step(const StepArgs &a, int n, unsigned ntiles, int lay, hipStream_t s)
{
    if (ntiles == 0) return;
    if (a.tile_rows == FLAT_TWO_ROWS) {
        if (lay == 0) hipLaunchKernelGGL(eh2_flat_kernel<0>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, a, n);
        else if (lay == 2) hipLaunchKernelGGL(eh2_flat_kernel<2>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, a, n);
        else hipLaunchKernelGGL(eh2_flat_kernel<3>, dim3(ntiles), dim3(FLAT_BLOCK), 0, s, a, n);
    } else if (lay == 1) {
        // tiles with r-layer rows, auxiliaries carried in registers: a
        // narrower block (TWO_CARRY_ROWS owned rows) leaves room for them
        hipLaunchKernelGGL((eh2_kernel<TWO_CARRY_ROWS, 3, true>), dim3(ntiles), dim3(64, TWO_CARRY_ROWS + 3, 1), 0, s,
                           a, n);
    } else if (lay == 4) {
        // r-layer band tiles without z-layer planes, auxiliaries carried:
        // the r-layer recursions only fit TWO_RBAND_ROWS rows at 3 waves per SIMD
        hipLaunchKernelGGL((eh2_kernel<TWO_RBAND_ROWS, 1, true>), dim3(ntiles), dim3(64, TWO_RBAND_ROWS + 3, 1), 0, s,
                           a, n);
    } else if (a.tile_rows == 13) launch_two_tr<13>(a, n, ntiles, lay, s);
    else launch_two_tr<5>(a, n, ntiles, lay, s);
}

void launch_three_step(const StepArgs &a, int n, unsigned ntiles, int lay, hipStream_t s)
{
    if (ntiles == 0) return;
    constexpr int TR = THREE_STEP_ROWS, TL = THREE_LAYER_ROWS;
    if (lay == 0) hipLaunchKernelGGL((eh3_kernel<TR, 0>), dim3(ntiles), dim3(64, TR + 5), 0, s, a, n);
    else if (lay == 2) hipLaunchKernelGGL((eh3_kernel<TR, 2>), dim3(ntiles), dim3(64, TR + 5), 0, s, a, n);
    else hipLaunchKernelGGL((eh3_kernel<TL, 3>), dim3(ntiles), dim3(64, TL + 5), 0, s, a, n);
}

unsigned tiles_split(const StepArgs &a, int BY)
{
    if (BY == FLAT_ROWS)
        return (((unsigned)a.nr * (unsigned)a.nphi + FLAT_BLOCK - 1) / FLAT_BLOCK) *
               (unsigned)((a.nz + a.kchunk - 1) / a.kchunk);
    return (unsigned)((a.nphi + BX - 1) / BX) * (unsigned)((a.nr + BY - 1) / BY) *
           (unsigned)((a.nz + a.kchunk - 1) / a.kchunk);
}

unsigned tiles_fused(const StepArgs &a, int TR)
{
    if (TR == FLAT_FUSED_ROWS) {
        const unsigned R = FLAT_BLOCK / a.nphi - 1;
        return (((unsigned)a.nr + R - 1) / R) * (unsigned)((a.nz + a.kchunk - 1) / a.kchunk);
    }
    return (unsigned)((a.nphi + FUSED_COLS - 1) / FUSED_COLS) * (unsigned)((a.nr + TR - 1) / TR) *
           (unsigned)((a.nz + a.kchunk - 1) / a.kchunk);
}

template <int BY>
void launch_batch_split(const BatchArgs &b, unsigned nblocks, int n_rel, hipStream_t s)
{
    hipLaunchKernelGGL(h_step_batch<BY>, dim3(nblocks), dim3(BX, BY), 0, s, b, n_rel);
    hipLaunchKernelGGL(e_step_batch<BY>, dim3(nblocks), dim3(BX, BY), 0, s, b, n_rel);
}

template <int TR>
void launch_batch_fused(const BatchArgs &b, unsigned nblocks, int n_rel, hipStream_t s)
{
    hipLaunchKernelGGL(eh_fused_batch<TR>, dim3(nblocks), dim3(64, TR + 1), 0, s, b, n_rel);
}

void launch_batch_step(const BatchArgs &b, unsigned nblocks, int tile_rows, bool fused, int n_rel, hipStream_t s)
{
    if (fused) {
        switch (tile_rows) {
        case FLAT_FUSED_ROWS:
            hipLaunchKernelGGL(eh_flat_batch, dim3(nblocks), dim3(FLAT_BLOCK), 0, s, b, n_rel);
            break;
        case 3: launch_batch_fused<3>(b, nblocks, n_rel, s); break;
        case 15: launch_batch_fused<15>(b, nblocks, n_rel, s); break;
        default: launch_batch_fused<7>(b, nblocks, n_rel, s); break;
        }
    } else {
        switch (tile_rows) {
        case FLAT_ROWS:
            hipLaunchKernelGGL(h_flat_batch, dim3(nblocks), dim3(FLAT_BLOCK), 0, s, b, n_rel);
            hipLaunchKernelGGL(e_flat_batch, dim3(nblocks), dim3(FLAT_BLOCK), 0, s, b, n_rel);
            break;
        case 1: launch_batch_split<1>(b, nblocks, n_rel, s); break;
        case 2: launch_batch_split<2>(b, nblocks, n_rel, s); break;
        case 8: launch_batch_split<8>(b, nblocks, n_rel, s); break;
        case 16: launch_batch_split<16>(b, nblocks, n_rel, s); break;
        default: launch_batch_split<4>(b, nblocks, n_rel, s); break;
        }
    }
}

void launch_advance_step(int *n_base, int by, hipStream_t s)
{
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, s, n_base, by);
}

void launch_set_int(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
}

void launch_fill(float2 *p, size_t n, hipStream_t s)
{
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

void launch_fill64(double2 *p, size_t n, hipStream_t s)
{
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

void launch_inv_eps64(double *ceps, const double *eps, size_t n, double dt, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(inv_eps64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ceps, eps, n, dt);
}

void launch_inv_eps(float *ceps, const float *eps, size_t n, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(inv_eps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ceps, eps, n, dt);
}

void launch_design_dt(float *ceps, const float *rho, size_t n, double eps_bg, double eps_hi, double dt,
                      hipStream_t s)
{
    hipLaunchKernelGGL(design_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ceps, rho, n, eps_bg,
                       eps_hi, dt);
}

void launch_seed_u(float2 *U, const float2 *Ep, int nr, int nphi, int nz, int pr0, int pr1, float dt,
                   hipStream_t s)
{
    hipLaunchKernelGGL(seed_u_kernel, dim3((nphi + 63) / 64, nr, nz), dim3(64), 0, s, U, Ep, nr, nphi, nz, pr0,
                       pr1, dt);
}

void launch_adjoint_pattern(float2 *pat, const float2 *g, const float2 *fac, int K, int nr, int nphi,
                            hipStream_t s)
{
    hipLaunchKernelGGL(adjoint_pattern_kernel, dim3((nphi + 63) / 64, nr, 2 * K), dim3(64), 0, s, pat, g, fac, K,
                       nr, nphi);
}

void launch_overlap(float *grad, const float2 *fwd, const float2 *adj, const float2 *wr, const float2 *wz,
                    int K, int nd, int nr, int nphi, float scale, hipStream_t s)
{
    hipLaunchKernelGGL(overlap_kernel, dim3((nphi + 63) / 64, nr, nd), dim3(64), 0, s, grad, fwd, adj, wr, wz, K,
                       nd, nr, nphi, scale);
}

void launch_watch(const WatchArgs &w, hipStream_t s)
{
    if (w.n == 0) return;
    size_t blocks = (w.n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(watch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, w);
}

void launch_nonfinite(const float2 *p, size_t n, int *flag, hipStream_t s)
{
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, flag);
}

}  // namespace zda
