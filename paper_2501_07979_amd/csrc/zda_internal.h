// zda_internal.h -- device-side parameter blocks shared by the gfx950 kernels
// and the host runtime of the ZDA zone library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/zda.h"

namespace zda {

// Complex sample type of a real type (interleaved re, im).
template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };

// Per-radial-row constants (index i, computed in FP64 on the host, rounded
// to R).  "int" = at r_i, "half" = at r_{i+1/2}.
template <typename R>
struct RowCoefT {
    R inv_rdphi_int, inv_rdphi_half;   // 1/(r dphi)
    R inv_2r_int, inv_2r_half;         // 1/(2 r)
    // divide-by-stretch recursions y = g1 x - g2 u, u <- c u + dt y
    R g1_s_int, g2_s_int, g1_s_half, g2_s_half;   // radial lengths l = dr (1 + sigma F)
    R g1_t_int, g2_t_int, g1_t_half, g2_t_half;   // radius ratio R / r = 1 + (Sigma/r) F
    R hz_c1, hz_c0;                    // Sigma_{i+1}/(r_{i+1/2} dr), Sigma_i/(r_{i+1/2} dr)
    R ez_c1, ez_c0;                    // Sigma_{i+1/2}/(r_i dr), Sigma_{i-1/2}/(r_i dr)
};
using RowCoef = RowCoefT<float>;

template <typename R>
struct ZCoefT {
    R g1_int, g2_int, g1_half, g2_half;   // axial lengths dz (1 + sigma_z F)
};
using ZCoef = ZCoefT<float>;

// Arguments of the update kernels (passed by value).  R = float is the
// production path; R = double instantiates the in-place kernel pair for the
// FP64 verification runs.
template <typename R>
struct StepArgsT {
    using C = typename CplxOf<R>::T;
    int nr, nphi, nz;
    int pr0, pr1, pz0, pz1;        // layer widths
    int dR, dZ;                    // slab thicknesses
    R dt, inv_dr, inv_dz;
    R cr, cz;                      // exp(-alpha dt)
    C seam_p, seam_m;              // exp(+i m tau), exp(-i m tau); 1 +- i m in a continuous zone
    int axis;                      // 1: row 0 is next to the axis (updated, no wall)
    // fields [nz][nr][nphi]
    C *Er, *Ep, *Ez, *Hr, *Hp, *Hz;
    const R *ceps;                 // dt/eps per cell
    C *auxR;                       // [10][nz][dR][nphi]
    C *auxZ;                       // [4][dZ][nr][nphi]
    const RowCoefT<R> *rows;       // [nr]
    const ZCoefT<R> *zrows;        // [nz]
    // source
    int k_src, n_prof;
    const C *pattern;              // [P][2][nr][nphi]
    const C *profile;              // [T][P]
    // DFT
    int K;
    const C *twiddle;              // [T][K]: dt e^{i w_k (n+1) dt}
    int k_mon;
    C *dft_plane;                  // [K][2][nr][nphi] or null
    int k0, k1;
    C *dft_vol;                    // [K][3][k1-k0][nr][nphi] or null
    int kchunk;                    // planes per z-chunk
    int tile_rows;                 // radial rows per block (1, 2, 4, 8, 16 split; 3, 7, 15 fused; 5, 13 two-step),
                                   // or a flat-mapping code (32, 33, 34)
    // fused step: fields and auxiliaries read from the set above, written here
    C *oEr, *oEp, *oEz, *oHr, *oHp, *oHz;
    C *oauxR, *oauxZ;
    int xcd_remap;                 // fused: contiguous tile ranges per XCD
    int nt_stores;                 // fused: non-temporal stores of the next buffer set
    // two-step launch: auxiliaries at the intermediate time level and the
    // linear indices of the tiles this launch covers
    C *mauxR, *mauxZ;
    const uint4 *tiles;            // {phi block, first row | rows << 16, kb | ke << 16, 0}
    // three-step launch: auxiliaries at the second intermediate time level
    C *m2auxR, *m2auxZ;
};
using StepArgs = StepArgsT<float>;
using StepArgs64 = StepArgsT<double>;

// Batched launch over many zones: per-zone argument blocks in device memory
// and the first block index of each zone (prefix sums of tile counts).
struct BatchArgs {
    const StepArgs *tab;
    const unsigned *prefix;
    int nzones;
    const int *n_base;             // device step offset added to the launch's step index
    int xcd_remap;
    const uint4 *tiles;            // two-step: tile descriptors, zone index in the fourth word
};

enum { AUX_HR_T, AUX_HP_S, AUX_HZ_S, AUX_HZ_T, AUX_V_HP,
       AUX_ER_T, AUX_EP_S, AUX_EZ_S, AUX_EZ_T, AUX_U_EP, N_AUX_R };
enum { ZAUX_HR, ZAUX_HP, ZAUX_ER, ZAUX_EP, N_AUX_Z };

void launch_h_step(const StepArgs &a, int n, hipStream_t s);
void launch_e_step(const StepArgs &a, int n, hipStream_t s);
// the in-place H and E kernels (4 rows x 64 phi cells per block) in FP64:
// fields, auxiliaries, coefficients, source and exit-plane DFT all double
void launch_h_step64(const StepArgs64 &a, int n, hipStream_t s);
void launch_e_step64(const StepArgs64 &a, int n, hipStream_t s);
void launch_fill64(double2 *p, size_t n, hipStream_t s);
// ceps = dt / eps elementwise in FP64
void launch_inv_eps64(double *ceps, const double *eps, size_t n, double dt, hipStream_t s);
void launch_fused_step(const StepArgs &a, int n, hipStream_t s);
// two leap-frog steps (n, n + 1) over the tiles listed in a.tiles; lay 0
// runs the instantiation without layer recursions (tiles whose computed rows
// and planes hold no layer cell), lay 2 with the flat mapping the one with
// the z-layer recursions only, any other value the one with the r- and
// z-layer recursions
void launch_two_step(const StepArgs &a, int n, unsigned ntiles, int lay, hipStream_t s);
// phi cells a tile owns.  56 (448 B) puts every tile's stores on 64 B
// boundaries of the row (for rows of a multiple of 8 cells), so no 64 B
// block of a field is written partly by two blocks (such blocks cost the
// memory a read-modify-write); 61 computes fewer halo cells per owned cell.
// The two-step tiles without layer cells are store-bound and take 56, the
// layer tiles (dearer per cell) 61; a two-step tile owns its phi cells, up to
// TR rows and a range of planes.
constexpr int two_step_cols(int lay) { return lay == 0 ? 56 : 61; }
// owned rows of the two-step tiles with r-layer rows whose step-one
// auxiliaries stay in registers (launch code lay = 1): 8-wavefront blocks
// of 195 VGPRs, two waves per SIMD (7 rows without the grouped loads of
// the level-n auxiliaries: 166 VGPRs, 3 waves per SIMD, 19 % slower)
constexpr int TWO_CARRY_ROWS = 5;
// owned rows of the carried two-step tiles of an r-layer band whose chunk
// holds no z-layer plane (launch code lay = 4): the r-layer recursions only,
// 10-wavefront blocks of 166 VGPRs, 3 waves per SIMD; taken for the bands
// that this cuts into fewer wavefront rows than TWO_CARRY_ROWS does
constexpr int TWO_RBAND_ROWS = 7;
// kinds of two-step tiles (lay codes 0..4)
constexpr int N_LAY = 5;
// Three-step kernel (three leap-frog steps per launch): the tile_rows code
// that selects it, the owned rows of its tiles without r-layer rows (16
// wavefronts, three halo rows below and two above) and of its r-layer band
// tiles (12 wavefronts), and its owned phi cells (56 on 64 B boundaries
// without layer cells; 59, all exact lanes, with them)
constexpr int THREE_STEP_ROWS = 11;
constexpr int THREE_LAYER_ROWS = 7;
constexpr int three_step_cols(int lay) { return lay == 0 ? 56 : 59; }
// three leap-frog steps (n, n + 1, n + 2) over the tiles listed in a.tiles;
// lay 0: no layer cell in the tile's computed rows and planes, lay 2: the
// z-layer recursions only, lay 3: r- and z-layer recursions (r-layer band
// tiles of THREE_LAYER_ROWS rows)
void launch_three_step(const StepArgs &a, int n, unsigned ntiles, int lay, hipStream_t s);
// a fused-step tile owns FUSED_COLS phi cells and TR rows
constexpr int FUSED_COLS = 56;
// tile_rows code of the in-place kernels with the flat (r, phi) mapping, its
// block size, and the widest zone (phi cells) that takes it by default
constexpr int FLAT_ROWS = 32;
// tile_rows code of the fused one-step kernel with the flat mapping (whole
// rows per block: needs nphi <= FLAT_FUSED_MAX_PHI)
constexpr int FLAT_FUSED_ROWS = 33;
constexpr int FLAT_FUSED_MAX_PHI = 64;
constexpr int FLAT_BLOCK_HOST = 256;
// tile_rows code of the two-step kernel with the flat mapping: a block holds
// FLAT_BLOCK_HOST / nphi whole rows, three of them the radial halo, so a tile
// owns flat_two_rows(nphi) rows and every phi cell (nphi <= FLAT_TWO_MAX_PHI)
constexpr int FLAT_TWO_ROWS = 34;
constexpr int FLAT_TWO_MAX_PHI = 32;
constexpr int flat_two_rows(int nphi) { return FLAT_BLOCK_HOST / nphi - 3; }
constexpr int NARROW_PHI = 16;
void launch_fill(float2 *p, size_t n, hipStream_t s);
// tiles of one zone for the split (BY rows) or fused (TR owned rows) kernels
unsigned tiles_split(const StepArgs &a, int BY);
unsigned tiles_fused(const StepArgs &a, int TR);
void launch_batch_step(const BatchArgs &b, unsigned nblocks, int tile_rows, bool fused, int n_rel, hipStream_t s);
// two steps of every zone of a batch over the tiles listed in b.tiles
void launch_batch_two(const BatchArgs &b, unsigned ntiles, int tile_rows, int lay, int n_rel, hipStream_t s);
void launch_advance_step(int *n_base, int by, hipStream_t s);
void launch_set_int(int *p, int v, hipStream_t s);
void launch_design_dt(float *ceps, const float *rho, size_t n, double eps_bg, double eps_hi, double dt,
                      hipStream_t s);
// ceps = dt / eps elementwise (eps may alias ceps; NULL eps means eps = 1)
void launch_inv_eps(float *ceps, const float *eps, size_t n, double dt, hipStream_t s);
void launch_seed_u(float2 *aux_u, const float2 *Ep, int nr, int nphi, int nz, int pr0, int pr1, float dt,
                   hipStream_t s);
void launch_adjoint_pattern(float2 *pat, const float2 *dFdE, const float2 *fac, int K, int nr, int nphi,
                            hipStream_t s);
void launch_overlap(float *grad, const float2 *fwd, const float2 *adj, const float2 *wr, const float2 *wz,
                    int K, int nd, int nr, int nphi, float scale, hipStream_t s);
void launch_nonfinite(const float2 *p, size_t n, int *flag, hipStream_t s);
// Divergence watchdog over up to six field arrays of n samples each (NULL
// entries skipped): *flag = 1 where a sample is not finite or |F|^2 is not
// below bound2.  The flag is never cleared here.
struct WatchArgs {
    const float2 *f[6];
    size_t n;
    int *flag;
    float bound2;
};
void launch_watch(const WatchArgs &w, hipStream_t s);

}  // namespace zda
