// Internal declarations shared by the liblbm translation units: the device
// descriptor of an instance, the tile work-list entry, the workspace layout
// and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// Columns of a tile: one 64-wide wavefront spans a tile row.
constexpr int TILE_X = 64;
// Threads per block: 4 wavefronts, one per row group of a tile.
constexpr int BLOCK = 256;
constexpr int ROW_GROUPS = BLOCK / TILE_X;
// Output columns of a two-step strip: a 64-wide wavefront spans the strip and
// three columns on each side.
constexpr int TWOSTEP_COLS = TILE_X - 6;
// Longest chunk of steps replayed from one captured graph; also the number of
// per-step wall-pressure slots an instance keeps.
constexpr int MAX_CHUNK = 256;
// Binary64 partial sums per tile written by the diagnostics kernel:
// mass, momentum x, momentum y, then one gas area per bubble.
constexpr int N_PARTIAL = 3 + LBM_MAX_BUBBLES;

// Per-instance constants in one precision, so that kernels read them as
// scalars instead of converting binary64 values in every lane.
template <typename T>
struct Consts {
    T RT, a, b4, two_over_G, mG;   // Eq. 15, Eq. 13 (2 / (G c^2)), -G of Eq. 7
    T rho_ref;                     // population shift reference
    T s_e, s_z, s_q, s_nu;         // rates of the relaxed moments (Eq. 2)
    T h_e, h_z, h_q, h_nu;         // 1 - s/2
    T li_e, li_z;                  // Li's term after (I - Lambda/2): s 0.75 eps
    // Relaxation (Eq. 3) and the scale c_k of the inverse transform folded
    // together, as increments: c_k (m*_k - m_k) = s_k c_k (m_eq_k - m_k)
    // + c_k (1 - s_k/2) S_k, with c = 1/36 (e, zeta), 1/12 (q), 1/4 (pxx,
    // pxy); the *_vf, *_li, *_f, *_xx and *_xy factors multiply the parts of
    // S_k of Eq. 14.
    T e_eq, e_vf, e_li;            // e row
    T z_eq, z_vf, z_li;            // zeta row
    T q_eq, q_f;                   // qx, qy rows
    T n_eq, n_xx, n_xy;            // pxx, pxy rows
};

// Device-visible description of one instance.  The host keeps a mirror and
// uploads it when it changes; kernels only read it, except the end-of-chunk
// kernel, which folds the per-step wall-pressure slots.
struct InstDev {
    void *f[2];                    // population buffers, 9 planes of ny*pitch
    void *psi;                     // ny*pitch pseudopotential values
    double *partials;              // N_PARTIAL * max_tiles binary64 partial sums
    int *flag;                     // [0] non-finite latch
    unsigned long long *wall_keys; // MAX_CHUNK per-step keys of the wall-row max of p
    unsigned long long *wall_run;  // [0] running max key, [1] its step
    double *result;                // reduced diagnostics (N_PARTIAL + 2 values)
    long long plane;               // ny * pitch
    long long step;                // steps taken before the current chunk
    int nx, ny, pitch, walls;
    int cur;                       // index of the buffer holding the current state
    int n_chunk;                   // steps this instance takes in the current chunk
    int tiles_x;                   // tiles per tile row for the current variant
    int n_bubbles;
    // Eq. 15 and Eq. 13 constants (two_over_G = 2 / (G c^2) with c = 1)
    double a, b4, RT, G, two_over_G;
    // relaxation rates of Eq. 2 that act on non-conserved moments
    double s_e, s_z, s_q, s_nu;
    // Li's term after (I - Lambda/2): s_e * 0.75 eps and s_zeta * 0.75 eps
    double li_e, li_z;
    double rho_l, rho_g;           // gas-fraction densities
    // Populations are stored shifted by the rest equilibrium of rho_ref:
    // g_a = f_a - w_a rho_ref (rho_ref representable in the storage precision)
    double rho_ref;
    // LBM_FP32_MIXED: Eqs. 15 and 13 in binary64 where mix_lo < rho - rho_ref
    // < mix_hi (the widened spinodal interval; empty at or above T_c)
    float mix_lo, mix_hi;
    double bx[LBM_MAX_BUBBLES], by[LBM_MAX_BUBBLES];
    Consts<float> cf;
    Consts<double> cd;
};

// One entry of the tile work-list.
struct Tile {
    int inst;
    int x0, y0;
    int tile_index;                // index of the tile within its instance
};

// Times the population buffers of an instance swap over n steps of a chunk:
// once per step, or, for the two-step variants (pairs != 0), once per launch,
// ceil(n / 2).
__host__ __device__ inline int buffer_flips(int n, int pairs) { return pairs ? (n + 1) >> 1 : n; }

// Kernel variants.  Two-pass variants (fused == 0) launch the psi pass and the
// force+collide+stream pass over tiles of TILE_X x (ROW_GROUPS * rows) sites,
// each thread taking `rows` rows.  Fused variants (fused == 1) launch one
// kernel per step over strips of TILE_X x rows sites that rebuild psi for the
// strip and its one-site ring on the fly.  Paired fused variants (fused == 2)
// do the same over strips of 2 * TILE_X x rows sites, two neighbouring sites
// per lane with two-element loads and stores; they need an even nx.  Two-step
// variants (fused == 3) launch one kernel per pair of steps over strips of
// TWOSTEP_COLS x rows sites.
struct Variant {
    int fused;
    int rows;
    const char *name;
};
extern const Variant kVariants[];
extern const int kNumVariants;

inline int tile_rows(int variant)
{
    return kVariants[variant].fused ? kVariants[variant].rows : ROW_GROUPS * kVariants[variant].rows;
}

inline int tile_cols(int variant)
{
    return kVariants[variant].fused == 2 ? 2 * TILE_X : (kVariants[variant].fused == 3 ? TWOSTEP_COLS : TILE_X);
}

inline bool two_step(int variant) { return kVariants[variant].fused == 3; }

inline bool variant_fits(int variant, int nx) { return kVariants[variant].fused != 2 || nx % 2 == 0; }

// Records, once per process, how many blocks of each fused kernel the
// current device holds at once (the fused kernels change their walk order
// when a whole grid fits).  Called where handles and batches are created,
// never under graph capture.
void prime_residency();
// Those blocks for one precision mode and variant (0: not known, or two-pass).
int resident_blocks(int prec, int variant);

// Kernels, launched on a stream.  prec is an lbm_precision.
hipError_t launch_psi_pass(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                           int ntiles, int s, hipStream_t st);
hipError_t launch_collide_stream(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                                 int ntiles, int s, hipStream_t st);
// write_through: the stores of the step write through L2 (see
// lbm_batch_set_write_through).
hipError_t launch_fused(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                        int s, hipStream_t st, int write_through = 0);
hipError_t launch_fused2(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                         int s, hipStream_t st);
// End of a chunk: folds the wall-pressure maxima, advances step and parity
// (buffer_flips(n, pairs)); with d_status, also copies each instance's latch
// to d_status[k].
// Two-step pass s: steps 2s and 2s + 1 of the chunk (only step 2s for an
// instance whose chunk ends there).
hipError_t launch_twostep(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                          int s, hipStream_t st, int write_through);
hipError_t launch_chunk_end(const InstDev *d_inst, int ninst, hipStream_t st, int *d_status = nullptr,
                            int pairs = 0);
hipError_t launch_init(int prec, const InstDev *d_inst, int slab_rows, const lbm_bubble *b, int nb,
                       double rho_l, double rho_g, double W, double delta, double noise_amp,
                       uint64_t seed, long long nsites, hipStream_t st);
hipError_t launch_init_density(int prec, const InstDev *d_inst, const double *rho, long long nsites,
                              hipStream_t st);
hipError_t launch_macros(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                         int ntiles, void *rho, void *ux, void *uy, double *p, hipStream_t st);
hipError_t launch_reduce(const InstDev *d_inst, int ntiles, hipStream_t st);
hipError_t launch_pack(int prec, const InstDev *d_inst, int nx, int ny, void *dense, int to_dense,
                       hipStream_t st);
hipError_t launch_reset_diag(const InstDev *d_inst, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t n, hipStream_t st);
// dst[0 .. n) = value (a kernel, so that it can be recorded in a graph)
hipError_t launch_fill_int(int *dst, int n, int value, hipStream_t st);

}  // namespace lbm
