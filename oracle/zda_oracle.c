/*
 * zda_oracle.c -- plain FP64 CPU oracle for one zone of zoned discrete
 * axisymmetry (ZDA): the cylindrical (r, phi, z) Yee FDTD time loop with the
 * Bloch seam, CPML in r and z, a general soft current source and on-the-fly
 * DFT monitors.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant generator with
 * the HIP library: every coefficient is recomputed here from its definition.
 *
 * Paper passages followed (arXiv 2501.07979):
 *  - Bloch form of the fields, eq. (1)-(2): the physical field is stored and
 *    the wedge boundary carries the phase exp(+-i m tau), tau = 2 pi / n.
 *  - Reduced Maxwell operator D_m, eq. (3)-(5): curl in cylindrical
 *    coordinates; with F = u exp(i m phi), D_m u = exp(-i m phi) curl F.
 *  - Section "Differentiable FDTD in cylindrical coordinates": staggered Yee
 *    grid, leap-frog in time, stretched-coordinate PML in r and z, r-PML
 *    regularised against divergence, DTFT monitors.
 *
 * Discretisation (the readings are listed in the design notes of the repo):
 *  cell (i, j, k): r_p = r_in + p dr for integer or half-integer p,
 *  phi_j = j dphi, dphi = 2 pi / (n_fold * nphi).
 *  E_r (i+1/2, j, k)   E_phi (i, j+1/2, k)   E_z (i, j, k+1/2)
 *  H_r (i, j+1/2, k+1/2)   H_phi (i+1/2, j, k+1/2)   H_z (i+1/2, j+1/2, k)
 *  All six arrays are complex, [nz][nr][nphi], phi fastest.  The box is PEC:
 *  E_r, E_phi vanish at k = 0 (and k = nz, outside storage); E_phi, E_z
 *  vanish at i = 0 (and i = nr).  H_r at i = 0 and H_z at k = 0 stay zero.
 *  Axis zone (axis = 1, r_in = dr/2, no inner layer): the axis is the row
 *  r_{-1/2} = 0, where nothing is stored.  The z components there are
 *  single-valued scalars that the Bloch condition F(phi + tau) =
 *  exp(i m tau) F(phi) forces to zero unless exp(i m tau) = 1, which axis
 *  zones must avoid; so row i = 0 is updated like any other row with
 *  H_z(-1/2) = 0, and the H_phi(-1/2) term of curlH_z carries the weight
 *  r_{-1/2} = 0.  H_r at i = 0 is updated.
 *  Continuous zone (n_fold = 0, nphi = 1, the n -> infinity limit of the
 *  first zone): fields carry exp(i m phi) exactly; the seam factors are
 *  1 +- i m with dphi = tau = 1, so the phi differences are exactly
 *  +-i m F / r and every component sits at phi = 0.
 *  Leap-frog (mu = 1, eps0 = mu0 = c = 1):
 *    H^{n+1/2} = H^{n-1/2} - dt * curlE(E^n)
 *    E^{n+1}   = E^n + (dt/eps) * (curlH(H^{n+1/2}) - J^{n+1/2})
 *  The radial derivative of (r F) is used in the algebraically identical
 *  split form dF/dr + avg(F)/r (no cancellation at large r in FP32 either).
 *  PML: complex coordinate stretching of the edge lengths and radii (see
 *  ora_create); in a layer a term x divided by a stretch (1 + s F) is
 *  advanced with one auxiliary recursion per term.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Public parameter block (mirrored by ctypes in oracle.py). */
typedef struct {
    double r_in, dr, dz, courant;
    int nr, nphi, nz, n_fold;
    int pml_r_in, pml_r_out, pml_z_lo, pml_z_hi;
    double pml_order, pml_sigma_max_r, pml_sigma_max_z, pml_alpha;
    int axis;                       /* 1: the zone contains the axis (r_in = dr / 2) */
} ora_params;

enum { ER = 0, EP = 1, EZ = 2, HR = 3, HP = 4, HZ = 5 };

/* auxiliary recursions of the r-layer (one complex per slab cell each) */
enum { A_HR_T, A_HP_S, A_HZ_S, A_HZ_T, A_U_EP,     /* H half-step */
       A_ER_T, A_EP_S, A_EZ_S, A_EZ_T, A_V_HP,     /* E half-step */
       N_AUX_R };
/* auxiliary recursions of the z-layer */
enum { Z_HR, Z_HP, Z_ER, Z_EP, N_AUX_Z };

typedef struct {
    ora_params p;
    double dt, dphi;
    size_t ncell;
    cplx *f[6];
    double *inv_eps;
    int dR, dZ;                 /* slab thicknesses (cells) */
    cplx *auxR[N_AUX_R];        /* [nz][dR][nphi] */
    cplx *auxZ[N_AUX_Z];        /* [dZ][nr][nphi] */
    double cr, cz;              /* exp(-alpha dt) of the r and z layers */
    /* per point, index 0 = integer position, 1 = half-integer position */
    double *sig_r[2], *sgt_r[2], *Sig_r[2];  /* sigma, sigma~ = Sigma/r, Sigma */
    double *sig_z[2];
} ora_zone;

static size_t cidx(const ora_zone *z, int k, int i, int j)
{
    return ((size_t)k * z->p.nr + i) * z->p.nphi + j;
}

/* slab row of cell index q along an axis with layers d0 (low) and d1 (high),
 * or -1 when q is not inside a layer */
static int slab_row(int q, int n, int d0, int d1)
{
    if (q < d0) return q;
    if (q >= n - d1) return d0 + (q - (n - d1));
    return -1;
}

/* graded conductivity sigma_max rho^order at coordinate p (cell units) */
static double grade(double p, int n, int d0, int d1, double order, double smax)
{
    double rho = 0.0;
    if (d0 > 0 && p < d0) rho = (d0 - p) / d0;
    else if (d1 > 0 && p > n - d1) rho = (p - (n - d1)) / d1;
    return rho > 0.0 ? smax * pow(rho, order) : 0.0;
}

void ora_destroy(ora_zone *z)
{
    if (!z) return;
    for (int c = 0; c < 6; c++) free(z->f[c]);
    for (int c = 0; c < N_AUX_R; c++) free(z->auxR[c]);
    for (int c = 0; c < N_AUX_Z; c++) free(z->auxZ[c]);
    for (int h = 0; h < 2; h++) { free(z->sig_r[h]); free(z->sgt_r[h]); free(z->Sig_r[h]); free(z->sig_z[h]); }
    free(z->inv_eps);
    free(z);
}

/*
 * Complex coordinate stretching (PML of the section on the cylindrical
 * solver).  With the causal one-pole filter F(w) = dt / (1 - c e^{i w dt}),
 * c = exp(-alpha dt) (the discrete 1/(alpha - i w)), every primal and dual
 * radial edge becomes l_p = dr (1 + sigma_p F), every radius becomes
 * R_p = r_p + Sigma_p F and every axial edge dz (1 + sigma_z F).  The curls
 * are circulations over stretched edges divided by stretched face areas, so
 * the scheme stays complex-symmetric under the stretched cell volumes.
 * Outer layer: Sigma is the running sum of sigma, R_{i+1} - R_i = l_{i+1/2}
 * exactly (the analytic continuation r~ = r + i Sigma / w).  Inner layer: the
 * continuation needs Sigma < 0, which diverges in time whatever the shift
 * alpha; the regularised layer uses |Sigma| (the radius is stretched into the
 * same half plane as on the outer side) while the radial lengths keep the
 * exact stretch.  All poles are then causal (sigma, Sigma >= 0).
 */
ora_zone *ora_create(const ora_params *p)
{
    if (!p || p->nr < 1 || p->nphi < 1 || p->nz < 1 || p->n_fold < 0) return NULL;
    if (p->n_fold == 0 && p->nphi != 1) return NULL;          /* continuous zone */
    if (p->axis && (p->pml_r_in != 0 || fabs(p->r_in - 0.5 * p->dr) > 1e-12 * p->dr)) return NULL;
    ora_zone *z = (ora_zone *)calloc(1, sizeof(ora_zone));
    if (!z) return NULL;
    z->p = *p;
    z->dt = p->courant * (p->dr < p->dz ? p->dr : p->dz);
    z->dphi = p->n_fold > 0 ? 2.0 * M_PI / ((double)p->n_fold * p->nphi) : 1.0;
    z->ncell = (size_t)p->nz * p->nr * p->nphi;
    z->dR = p->pml_r_in + p->pml_r_out;
    z->dZ = p->pml_z_lo + p->pml_z_hi;
    int ok = 1;
    for (int c = 0; c < 6; c++) ok &= (z->f[c] = (cplx *)calloc(z->ncell, sizeof(cplx))) != NULL;
    z->inv_eps = (double *)malloc(z->ncell * sizeof(double));
    ok &= z->inv_eps != NULL;
    if (z->dR > 0)
        for (int c = 0; c < N_AUX_R; c++)
            ok &= (z->auxR[c] = (cplx *)calloc((size_t)p->nz * z->dR * p->nphi, sizeof(cplx))) != NULL;
    if (z->dZ > 0)
        for (int c = 0; c < N_AUX_Z; c++)
            ok &= (z->auxZ[c] = (cplx *)calloc((size_t)z->dZ * p->nr * p->nphi, sizeof(cplx))) != NULL;
    for (int h = 0; h < 2; h++) {
        ok &= (z->sig_r[h] = (double *)calloc(p->nr + 1, sizeof(double))) != NULL;
        ok &= (z->sgt_r[h] = (double *)calloc(p->nr + 1, sizeof(double))) != NULL;
        ok &= (z->Sig_r[h] = (double *)calloc(p->nr + 1, sizeof(double))) != NULL;
        ok &= (z->sig_z[h] = (double *)calloc(p->nz + 1, sizeof(double))) != NULL;
    }
    if (!ok) { ora_destroy(z); return NULL; }
    for (size_t c = 0; c < z->ncell; c++) z->inv_eps[c] = 1.0;

    const int nr = p->nr, nz = p->nz, d0 = p->pml_r_in, d1 = p->pml_r_out;
    double smr = p->pml_sigma_max_r > 0 ? p->pml_sigma_max_r : 0.8 * (p->pml_order + 1.0) / p->dr;
    double smz = p->pml_sigma_max_z > 0 ? p->pml_sigma_max_z : 0.8 * (p->pml_order + 1.0) / p->dz;
    for (int h = 0; h < 2; h++) {
        for (int i = 0; i <= nr; i++) z->sig_r[h][i] = grade(i + 0.5 * h, nr, d0, d1, p->pml_order, smr);
        for (int k = 0; k <= nz; k++) z->sig_z[h][k] = grade(k + 0.5 * h, nz, p->pml_z_lo, p->pml_z_hi, p->pml_order, smz);
    }
    /* Sigma: zero between the layers; integer points accumulate sigma of the
     * half points between them, half points that of the integer points. */
    for (int i = 0; i <= nr; i++) { z->Sig_r[0][i] = 0.0; z->Sig_r[1][i] = 0.0; }
    for (int i = nr - d1 + 1; i <= nr && d1 > 0; i++)
        z->Sig_r[0][i] = z->Sig_r[0][i - 1] + p->dr * z->sig_r[1][i - 1];
    for (int i = nr - d1; i <= nr && d1 > 0; i++)
        z->Sig_r[1][i] = (i > 0 ? z->Sig_r[1][i - 1] : 0.0) + p->dr * z->sig_r[0][i];
    /* inner layer: the exact continuation would subtract here (Sigma < 0)
     * and diverges in time; the regularised radius grows inwards instead */
    for (int i = d0 - 1; i >= 0 && d0 > 0; i--)
        z->Sig_r[0][i] = z->Sig_r[0][i + 1] + p->dr * z->sig_r[1][i];
    for (int i = d0 - 1; i >= 0 && d0 > 0; i--)
        z->Sig_r[1][i] = z->Sig_r[1][i + 1] + p->dr * z->sig_r[0][i + 1];
    double worst = 0.0;
    for (int h = 0; h < 2; h++)
        for (int i = 0; i <= nr; i++) {
            double r = p->r_in + (i + 0.5 * h) * p->dr;
            z->sgt_r[h][i] = z->Sig_r[h][i] / r;
            if (-z->sgt_r[h][i] > worst) worst = -z->sgt_r[h][i];
        }
    double alpha_r = p->pml_alpha + 2.0 * worst;
    z->cr = exp(-alpha_r * z->dt);
    z->cz = exp(-p->pml_alpha * z->dt);
    return z;
}

double ora_dt(const ora_zone *z) { return z->dt; }

/* threads the time loop uses */
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Layer constants: which = 0 r-integer, 1 r-half, 2 z-integer, 3 z-half.
 * sig, sgt (sigma~ = Sigma/r, zero for z) and the pole c = exp(-alpha dt). */
void ora_get_layer(const ora_zone *z, int which, double *sig, double *sgt, double *c)
{
    int h = which & 1;
    if (which < 2) {
        memcpy(sig, z->sig_r[h], z->p.nr * sizeof(double));
        memcpy(sgt, z->sgt_r[h], z->p.nr * sizeof(double));
        *c = z->cr;
    } else {
        memcpy(sig, z->sig_z[h], z->p.nz * sizeof(double));
        memset(sgt, 0, z->p.nz * sizeof(double));
        *c = z->cz;
    }
}

void ora_set_eps(ora_zone *z, const float *eps)
{
    for (size_t c = 0; c < z->ncell; c++) z->inv_eps[c] = 1.0 / (double)eps[c];
}

/* FP64 permittivity, for finite-difference checks below FP32 resolution */
void ora_set_eps64(ora_zone *z, const double *eps)
{
    for (size_t c = 0; c < z->ncell; c++) z->inv_eps[c] = 1.0 / eps[c];
}

void ora_reset(ora_zone *z)
{
    for (int c = 0; c < 6; c++) memset(z->f[c], 0, z->ncell * sizeof(cplx));
    for (int c = 0; c < N_AUX_R; c++)
        if (z->auxR[c]) memset(z->auxR[c], 0, (size_t)z->p.nz * z->dR * z->p.nphi * sizeof(cplx));
    for (int c = 0; c < N_AUX_Z; c++)
        if (z->auxZ[c]) memset(z->auxZ[c], 0, (size_t)z->dZ * z->p.nr * z->p.nphi * sizeof(cplx));
}

void ora_set_field(ora_zone *z, int comp, const cplx *src) { memcpy(z->f[comp], src, z->ncell * sizeof(cplx)); }
void ora_get_field(const ora_zone *z, int comp, cplx *dst) { memcpy(dst, z->f[comp], z->ncell * sizeof(cplx)); }

/* y = x / (1 + s F): with u = F y, y^n + s (c u^{n-1} + dt y^n) = x^n.
 * Identity when the point is outside the layer (aux == NULL). */
static cplx divide_stretch(cplx x, cplx *aux, double s, double c, double dt)
{
    if (!aux) return x;
    cplx y = (x - s * c * (*aux)) / (1.0 + s * dt);
    *aux = c * (*aux) + dt * y;
    return y;
}

/* H half-step: H^{n+1/2} = H^{n-1/2} - dt curlE(E^n) (eq. 3 with mu = 1). */
static void step_h(ora_zone *z, cplx seam_p)
{
    const ora_params *p = &z->p;
    const int nr = p->nr, np = p->nphi, nz = p->nz;
    const double dr = p->dr, dz = p->dz, dph = z->dphi, dt = z->dt;
    cplx *Er = z->f[ER], *Ep = z->f[EP], *Ez = z->f[EZ];
    cplx *Hr = z->f[HR], *Hp = z->f[HP], *Hz = z->f[HZ];
    /* U = F E_phi at the integer radial points of the r-layer, advanced first
     * because both neighbouring H_z rows read it */
    if (z->dR > 0) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; k++)
            for (int i = 0; i < nr; i++) {
                int ir = slab_row(i, nr, p->pml_r_in, p->pml_r_out);
                if (ir < 0) continue;
                for (int j = 0; j < np; j++) {
                    cplx *u = &z->auxR[A_U_EP][((size_t)k * z->dR + ir) * np + j];
                    *u = z->cr * (*u) + dt * Ep[cidx(z, k, i, j)];
                }
            }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        int kz = slab_row(k, nz, p->pml_z_lo, p->pml_z_hi);
        for (int i = 0; i < nr; i++) {
            int ir = slab_row(i, nr, p->pml_r_in, p->pml_r_out);
            int ir1 = i + 1 < nr ? slab_row(i + 1, nr, p->pml_r_in, p->pml_r_out) : -1;
            double r_i = p->r_in + i * dr, r_h = p->r_in + (i + 0.5) * dr;
            for (int j = 0; j < np; j++) {
                size_t c = cidx(z, k, i, j);
                size_t sr = ir >= 0 ? ((size_t)k * z->dR + ir) * np + j : 0;
                size_t sz = kz >= 0 ? ((size_t)kz * nr + i) * np + j : 0;
                /* neighbours with the PEC box and the Bloch seam */
                cplx ez_jp = j + 1 < np ? Ez[c + 1] : seam_p * Ez[cidx(z, k, i, 0)];
                cplx er_jp = j + 1 < np ? Er[c + 1] : seam_p * Er[cidx(z, k, i, 0)];
                cplx ep_kp = k + 1 < nz ? Ep[cidx(z, k + 1, i, j)] : 0.0;
                cplx er_kp = k + 1 < nz ? Er[cidx(z, k + 1, i, j)] : 0.0;
                cplx ez_ip = i + 1 < nr ? Ez[cidx(z, k, i + 1, j)] : 0.0;
                cplx ep_ip = i + 1 < nr ? Ep[cidx(z, k, i + 1, j)] : 0.0;
                /* H_r at (i, j+1/2, k+1/2): dEz/dphi / R_i - dEphi/dz / s_z */
                if (i > 0 || p->axis) {
                    cplx t1 = (ez_jp - Ez[c]) / (r_i * dph);
                    cplx t2 = (ep_kp - Ep[c]) / dz;
                    t1 = divide_stretch(t1, ir >= 0 ? &z->auxR[A_HR_T][sr] : NULL, z->sgt_r[0][i], z->cr, dt);
                    t2 = divide_stretch(t2, kz >= 0 ? &z->auxZ[Z_HR][sz] : NULL, z->sig_z[1][k], z->cz, dt);
                    Hr[c] -= dt * (t1 - t2);
                }
                /* H_phi at (i+1/2, j, k+1/2): dEr/dz / s_z - dEz/dr / s_r */
                {
                    cplx t1 = (er_kp - Er[c]) / dz;
                    cplx t2 = (ez_ip - Ez[c]) / dr;
                    t1 = divide_stretch(t1, kz >= 0 ? &z->auxZ[Z_HP][sz] : NULL, z->sig_z[1][k], z->cz, dt);
                    t2 = divide_stretch(t2, ir >= 0 ? &z->auxR[A_HP_S][sr] : NULL, z->sig_r[1][i], z->cr, dt);
                    Hp[c] -= dt * (t1 - t2);
                }
                /* H_z at (i+1/2, j+1/2, k): [d(R Ephi)/dr / l - dEr/dphi] / R */
                if (k > 0) {
                    cplx t = (ep_ip - Ep[c]) / dr + (ep_ip + Ep[c]) / (2.0 * r_h);
                    if (ir >= 0) {
                        cplx u0 = z->auxR[A_U_EP][sr];
                        cplx u1 = ir1 >= 0 ? z->auxR[A_U_EP][((size_t)k * z->dR + ir1) * np + j] : 0.0;
                        double S1 = i + 1 < nr ? z->Sig_r[0][i + 1] : 0.0;
                        t += (S1 * u1 - z->Sig_r[0][i] * u0) / (r_h * dr);
                        t = divide_stretch(t, &z->auxR[A_HZ_S][sr], z->sig_r[1][i], z->cr, dt);
                    }
                    t -= (er_jp - Er[c]) / (r_h * dph);
                    t = divide_stretch(t, ir >= 0 ? &z->auxR[A_HZ_T][sr] : NULL, z->sgt_r[1][i], z->cr, dt);
                    Hz[c] -= dt * t;
                }
            }
        }
    }
}

/* E half-step: E^{n+1} = E^n + (dt/eps) (curlH(H^{n+1/2}) - J^{n+1/2}) (eq. 4).
 * Jr, Jp: source current on plane k_src ([nr][nphi] each) or NULL. */
static void step_e(ora_zone *z, cplx seam_m, int k_src, const cplx *Jr, const cplx *Jp)
{
    const ora_params *p = &z->p;
    const int nr = p->nr, np = p->nphi, nz = p->nz;
    const double dr = p->dr, dz = p->dz, dph = z->dphi, dt = z->dt;
    cplx *Er = z->f[ER], *Ep = z->f[EP], *Ez = z->f[EZ];
    cplx *Hr = z->f[HR], *Hp = z->f[HP], *Hz = z->f[HZ];
    /* V = F H_phi at the half radial points of the r-layer */
    if (z->dR > 0) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; k++)
            for (int i = 0; i < nr; i++) {
                int ir = slab_row(i, nr, p->pml_r_in, p->pml_r_out);
                if (ir < 0) continue;
                for (int j = 0; j < np; j++) {
                    cplx *v = &z->auxR[A_V_HP][((size_t)k * z->dR + ir) * np + j];
                    *v = z->cr * (*v) + dt * Hp[cidx(z, k, i, j)];
                }
            }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        int kz = slab_row(k, nz, p->pml_z_lo, p->pml_z_hi);
        for (int i = 0; i < nr; i++) {
            int ir = slab_row(i, nr, p->pml_r_in, p->pml_r_out);
            int irm = i > 0 ? slab_row(i - 1, nr, p->pml_r_in, p->pml_r_out) : -1;
            double r_i = p->r_in + i * dr, r_h = p->r_in + (i + 0.5) * dr;
            for (int j = 0; j < np; j++) {
                size_t c = cidx(z, k, i, j);
                size_t sr = ir >= 0 ? ((size_t)k * z->dR + ir) * np + j : 0;
                size_t sz = kz >= 0 ? ((size_t)kz * nr + i) * np + j : 0;
                double ce = dt * z->inv_eps[c];
                cplx hz_jm = j > 0 ? Hz[c - 1] : seam_m * Hz[cidx(z, k, i, np - 1)];
                cplx hr_jm = j > 0 ? Hr[c - 1] : seam_m * Hr[cidx(z, k, i, np - 1)];
                int src = (k == k_src) && Jr;
                /* E_r at (i+1/2, j, k): dHz/dphi / R - dHphi/dz / s_z */
                if (k > 0) {
                    cplx t1 = (Hz[c] - hz_jm) / (r_h * dph);
                    cplx t2 = (Hp[c] - Hp[cidx(z, k - 1, i, j)]) / dz;
                    t1 = divide_stretch(t1, ir >= 0 ? &z->auxR[A_ER_T][sr] : NULL, z->sgt_r[1][i], z->cr, dt);
                    t2 = divide_stretch(t2, kz >= 0 ? &z->auxZ[Z_ER][sz] : NULL, z->sig_z[0][k], z->cz, dt);
                    cplx j_r = src ? Jr[(size_t)i * np + j] : 0.0;
                    Er[c] += ce * (t1 - t2 - j_r);
                }
                /* E_phi at (i, j+1/2, k): dHr/dz / s_z - dHz/dr / s_r (H_z on the axis is 0) */
                if (k > 0 && (i > 0 || p->axis)) {
                    cplx hz_im = i > 0 ? Hz[cidx(z, k, i - 1, j)] : 0.0;
                    cplx t1 = (Hr[c] - Hr[cidx(z, k - 1, i, j)]) / dz;
                    cplx t2 = (Hz[c] - hz_im) / dr;
                    t1 = divide_stretch(t1, kz >= 0 ? &z->auxZ[Z_EP][sz] : NULL, z->sig_z[0][k], z->cz, dt);
                    t2 = divide_stretch(t2, ir >= 0 ? &z->auxR[A_EP_S][sr] : NULL, z->sig_r[0][i], z->cr, dt);
                    cplx j_p = src ? Jp[(size_t)i * np + j] : 0.0;
                    Ep[c] += ce * (t1 - t2 - j_p);
                }
                /* E_z at (i, j, k+1/2): [d(R Hphi)/dr / l - dHr/dphi] / R
                 * (on the axis row the H_phi(-1/2) term has weight r = 0) */
                if (i > 0 || p->axis) {
                    cplx hp_im = i > 0 ? Hp[cidx(z, k, i - 1, j)] : 0.0;
                    cplx t = (Hp[c] - hp_im) / dr + (Hp[c] + hp_im) / (2.0 * r_i);
                    if (ir >= 0) {
                        cplx v1 = z->auxR[A_V_HP][sr];
                        cplx v0 = irm >= 0 ? z->auxR[A_V_HP][((size_t)k * z->dR + irm) * np + j] : 0.0;
                        double S0 = i > 0 ? z->Sig_r[1][i - 1] : 0.0;
                        t += (z->Sig_r[1][i] * v1 - S0 * v0) / (r_i * dr);
                        t = divide_stretch(t, &z->auxR[A_EZ_S][sr], z->sig_r[0][i], z->cr, dt);
                    }
                    t -= (Hr[c] - hr_jm) / (r_i * dph);
                    t = divide_stretch(t, ir >= 0 ? &z->auxR[A_EZ_T][sr] : NULL, z->sgt_r[0][i], z->cr, dt);
                    Ez[c] += ce * t;
                }
            }
        }
    }
}

/*
 * Run nsteps leap-frog steps from the current state (no reset).
 *  m        Bloch angular momentum used for the seam phase exp(+-i m tau)
 *  n_start  global index of the first step (sets the DFT and source time)
 *  source   P profiles: J^{n+1/2}(x) = sum_p pat[p](x) * prof[p][n]
 *           pat: [P][2][nr][nphi] complex (J_r, J_phi on plane k_src)
 *           prof: [P][nsteps] complex
 *  DFT      Ehat_k += dt * exp(i w_k N dt) E^N for N = n_start+n+1 (section on
 *           the adjoint: DTFT monitors).  plane: [K][2][nr][nphi] (E_r, E_phi
 *           at k_mon); vol: [K][3][k1-k0][nr][nphi] (E_r, E_phi, E_z).
 * Returns 0, or -1 on bad arguments.
 */
int ora_run(ora_zone *z, int m, int nsteps, long n_start,
            int P, const cplx *pat, const cplx *prof, int k_src,
            int K, const double *omega,
            int k_mon, cplx *dft_plane,
            int k0, int k1, cplx *dft_vol)
{
    const ora_params *p = &z->p;
    const int nr = p->nr, np = p->nphi;
    const size_t plane = (size_t)nr * np;
    if (P > 0 && (k_src < 1 || k_src >= p->nz || !pat || !prof)) return -1;
    if (dft_plane && (k_mon < 0 || k_mon >= p->nz)) return -1;
    if (dft_vol && (k0 < 0 || k1 > p->nz || k0 >= k1)) return -1;
    cplx seam_p, seam_m;
    if (p->n_fold > 0) {
        double tau = 2.0 * M_PI / p->n_fold;
        seam_p = cexp(I * m * tau);
        seam_m = cexp(-I * m * tau);
    } else {                        /* continuous zone: exact i m derivative */
        seam_p = 1.0 + I * m;
        seam_m = 1.0 - I * m;
    }
    if (p->axis && cabs(seam_p - 1.0) < 1e-12) return -1;   /* axis scalars would not vanish */
    cplx *Jr = NULL, *Jp = NULL;
    if (P > 0) {
        Jr = (cplx *)malloc(plane * sizeof(cplx));
        Jp = (cplx *)malloc(plane * sizeof(cplx));
        if (!Jr || !Jp) { free(Jr); free(Jp); return -1; }
    }
    cplx *tw = (cplx *)malloc((K > 0 ? K : 1) * sizeof(cplx));
    for (int n = 0; n < nsteps; n++) {
        step_h(z, seam_p);
        if (P > 0) {
            for (size_t q = 0; q < plane; q++) { Jr[q] = 0.0; Jp[q] = 0.0; }
            for (int s = 0; s < P; s++) {
                cplx g = prof[(size_t)s * nsteps + n];
                const cplx *pr = pat + (size_t)s * 2 * plane;
                for (size_t q = 0; q < plane; q++) { Jr[q] += pr[q] * g; Jp[q] += pr[plane + q] * g; }
            }
        }
        step_e(z, seam_m, k_src, Jr, Jp);
        long N = n_start + n + 1;
        for (int kk = 0; kk < K; kk++) tw[kk] = z->dt * cexp(I * omega[kk] * (double)N * z->dt);
        if (dft_plane) {
            for (int kk = 0; kk < K; kk++) {
                cplx *o = dft_plane + (size_t)kk * 2 * plane;
                const cplx *er = z->f[ER] + cidx(z, k_mon, 0, 0);
                const cplx *ep = z->f[EP] + cidx(z, k_mon, 0, 0);
                for (size_t q = 0; q < plane; q++) { o[q] += tw[kk] * er[q]; o[plane + q] += tw[kk] * ep[q]; }
            }
        }
        if (dft_vol) {
            int nd = k1 - k0;
#pragma omp parallel for schedule(static)
            for (int kd = 0; kd < nd; kd++)
                for (int kk = 0; kk < K; kk++)
                    for (int comp = 0; comp < 3; comp++) {
                        cplx *o = dft_vol + (((size_t)kk * 3 + comp) * nd + kd) * plane;
                        const cplx *f = z->f[comp] + cidx(z, k0 + kd, 0, 0);
                        for (size_t q = 0; q < plane; q++) o[q] += tw[kk] * f[q];
                    }
        }
    }
    free(tw); free(Jr); free(Jp);
    return 0;
}
