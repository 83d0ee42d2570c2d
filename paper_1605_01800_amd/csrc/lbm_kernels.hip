// gfx950 kernels of the D2Q9 pseudopotential MRT lattice Boltzmann timestep
// (Shan et al., arXiv:1605.01800).
//
// Populations are kept post-streaming in structure-of-arrays form: plane a
// holds f_a for every site, rows of `pitch` elements (a multiple of 64), so a
// 64-wide wavefront reads one row segment of one plane with one coalesced
// access.  A step is two passes over a work-list of 64 x (4*RY) tiles:
//
//   psi pass               rho = sum_a f_a, p (Eq. 15), psi (Eq. 13); stores psi
//   force+collide+stream   stages the tile's psi plus a one-site halo in LDS,
//                          then per site: F (Eq. 7), v (Eq. 6), moments and
//                          equilibria (Eq. 4), Li's source (Eq. 14), relaxation
//                          (Eq. 3), f* = M^-1 m*, and pushes f*_a to x + e_a in
//                          the other buffer (Eq. 5) or, through a wall, back to
//                          the same site as the opposite population.
//
// The moment transform is applied per site with its integer structure written
// out (it is a sparse 9x9 map, not a contraction, so it stays on the vector
// ALUs).  Blocks are mapped to tiles so that each of the eight XCDs works on a
// contiguous run of tiles, which keeps halo re-reads in that XCD's L2.
#include <math.h>

#include <atomic>
#include <mutex>

#include "lbm_internal.h"
#include "lbm_rounding.h"

namespace lbm {

const Variant kVariants[] = {
    {0, 1, "2pass-64x4"},    {0, 2, "2pass-64x8"},    {0, 4, "2pass-64x16"},   {0, 8, "2pass-64x32"},
    {1, 16, "fused-64x16"},  {1, 32, "fused-64x32"},  {1, 64, "fused-64x64"},  {1, 128, "fused-64x128"},
    {2, 16, "fused2-128x16"}, {2, 32, "fused2-128x32"}, {2, 64, "fused2-128x64"},
    {3, 16, "twostep-58x16"}, {3, 24, "twostep-58x24"}, {3, 32, "twostep-58x32"}, {3, 48, "twostep-58x48"},
    {3, 64, "twostep-58x64"}};
const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

namespace {

constexpr int NXCD = 8;

// Population and psi buffers are reached through descriptors, so the compiler
// sees generic pointers and would emit flat memory instructions, which also
// count against the LDS wait counter and serialise the LDS reads behind the
// outstanding population loads.  Casting to the global address space gives
// global loads and stores.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> global_ptr(void *p)
{
    return (gptr<T>)p;
}

// A wavefront always works on one row, so the address of a population is a
// wave-uniform row base (plane base + row offset, kept in scalar registers)
// plus a per-lane byte offset below 4 GiB (every plane is under 4 GiB, checked
// when an instance is created).  Written this way the loads and stores take
// the scalar-base + 32-bit-offset form and all nine planes share one offset
// register, instead of costing two address registers per access.
//
// The compiler tends to fold the scalar row offset into a per-lane 64-bit
// address instead (one extra vector add per access); passing the row base
// through an empty register-only asm statement that keeps it in scalar
// registers prevents that.  Callers guarantee that row_base is the same in
// every lane of the wavefront.
template <typename P>
__device__ __forceinline__ P scalar_base(P p)
{
    asm("" : "+s"(p));
    return p;
}

// Likewise the 32-bit lane offset is passed through an empty asm statement at
// every use, so that its widening to 64 bits stays next to the access (where
// it folds into the addressing mode) rather than being hoisted out as a
// 64-bit register pair.
__device__ __forceinline__ unsigned lane_offset(unsigned o)
{
    asm("" : "+v"(o));
    return o;
}

template <typename T>
__device__ __forceinline__ T ld(gptr<const char> row_base, unsigned lane_off)
{
    return *(gptr<const T>)(scalar_base(row_base) + lane_offset(lane_off));
}

template <typename T>
__device__ __forceinline__ void st(gptr<char> row_base, unsigned lane_off, T v)
{
    *(gptr<T>)(scalar_base(row_base) + lane_offset(lane_off)) = v;
}

// Store that, with WT, is a relaxed agent-scope atomic store: a vector store
// that writes through the XCD's L2, so the line is not left dirty there.
template <typename T, bool WT>
__device__ __forceinline__ void stw(gptr<char> row_base, unsigned lane_off, T v)
{
    gptr<T> p = (gptr<T>)(scalar_base(row_base) + lane_offset(lane_off));
    if constexpr (WT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// Load whose address differs across the wavefront.
template <typename T>
__device__ __forceinline__ T ld_lane(gptr<const char> base, unsigned long long off)
{
    return *(gptr<const T>)(base + off);
}

// Index of the calling thread's wavefront, as a scalar.
__device__ __forceinline__ int wave_index()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x / TILE_X);
}

// x / 6 as x * hi + x * lo, with hi + lo the reciprocal to twice the
// working precision: one rounding of a nearly exact quotient, so the result is
// the correctly rounded quotient except in rare near-ties and, unlike x * hi
// alone, has no systematic bias.
template <typename T>
struct Sixth;
template <>
struct Sixth<float> {
    static constexpr float r6_hi = 0x1.555556p-3f, r6_lo = -0x1.555556p-28f;
};
template <>
struct Sixth<double> {
    static constexpr double r6_hi = 0x1.5555555555555p-3, r6_lo = 0x1.5555555555555p-57;
};

template <typename T>
__device__ __forceinline__ T div6(T x)
{
    return fma(x, Sixth<T>::r6_hi, x * Sixth<T>::r6_lo);
}

// Block b of a grid of nblocks (a multiple of NXCD) runs tile xcd_tile(b):
// consecutive dispatch slots of one XCD take consecutive tiles.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks / NXCD;
    return (b % NXCD) * per + b / NXCD;
}

// Source buffer of step s of the current chunk; s < 0 means the current state.
__device__ __forceinline__ int src_buffer(const InstDev &d, int s)
{
    return s < 0 ? d.cur : ((d.cur + s) & 1);
}

// Populations are stored as g_a = f_a - w_a rho_ref, the deviation from the
// rest equilibrium of a reference density (the liquid density of the run).
// In uniform regions every site computes nearly the same numbers, so rounding
// errors add up coherently instead of averaging out; with the shift they act on
// deviations instead of on the populations themselves, which makes them about
// |f - w rho_ref| / |f| smaller (three orders of magnitude in the liquid).
//
// sum_a g_a = rho - rho_ref, always in this order.
//
// Mirror-symmetric rounding.  Every sum over populations below is written
// as a tree that a reflection of the lattice (x -> -x swaps 1 <-> 3, 5 <-> 6,
// 7 <-> 8; y -> -y swaps 2 <-> 4, 5 <-> 8, 6 <-> 7) maps onto itself, up to
// the order of the two operands of an addition (which does not change a
// rounded sum) and up to an exact sign change.  A state that is symmetric
// under a reflection then stays symmetric bit for bit, as the exact
// dynamics does: a disc or slab at the centre of a periodic grid cannot
// drift by accumulating rounding errors that favour one side.  (Written in
// population order instead, the binary32 path moved such interfaces by up to
// 6e-3 sites in 40,000 steps, which shows as 1.7e-3 of the density range at
// the interface.)
template <typename T>
__device__ __forceinline__ T density(const T v[9])
{
    return (((v[1] + v[3]) + (v[2] + v[4])) + ((v[5] + v[7]) + (v[6] + v[8]))) + v[0];
}

// Momentum sums of Eq. 6 in mirror-symmetric form: an x reflection negates
// jx exactly and leaves jy unchanged, a y reflection the reverse.
template <typename T>
__device__ __forceinline__ T momentum_x(const T v[9])
{
    return (v[1] - v[3]) + ((v[5] + v[8]) - (v[6] + v[7]));
}

template <typename T>
__device__ __forceinline__ T momentum_y(const T v[9])
{
    return (v[2] - v[4]) + ((v[5] + v[6]) - (v[7] + v[8]));
}

// 1/x and sqrt(x).  In binary64 correctly rounded.  In binary32 the hardware
// instructions (at most one unit in the last place off) replace the longer
// correctly rounded sequences: none of these quotients enters a conserved
// moment (div6 handles those), so the extra error is unbiased noise
// well below the binary32 path's own rounding.
template <typename T>
__device__ __forceinline__ T recip(T x)
{
    return T(1) / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}
template <typename T>
__device__ __forceinline__ T root(T x)
{
    return sqrt(x);
}
template <>
__device__ __forceinline__ float root<float>(float x)
{
    return __builtin_amdgcn_sqrtf(x);
}

// Carnahan-Starling pressure, Eq. 15, with eta = (b/4) rho.
//
// Here and in the site arithmetic below, contraction of products into fused
// multiply-adds is switched off and every fma is written out: where a sum has
// two products, or a product feeds a value with other uses, the compiler's
// choice of what to fuse otherwise depends on the surrounding kernel, and the
// kernel variants would round differently.
template <typename T>
__device__ __forceinline__ T eos_pressure(T rho, T RT, T a, T b4)
{
#pragma clang fp contract(off)
    const T eta = b4 * rho;
    const T om = T(1) - eta;
    const T num = fma(eta, fma(eta, T(1) - eta, T(1)), T(1));
    return fma(rho * RT * num, recip(om * om * om), -(a * rho * rho));
}

// The instance constants in the working precision.
template <typename T>
__device__ __forceinline__ const Consts<T> &consts(const InstDev &d);
template <>
__device__ __forceinline__ const Consts<float> &consts<float>(const InstDev &d)
{
    return d.cf;
}
template <>
__device__ __forceinline__ const Consts<double> &consts<double>(const InstDev &d)
{
    return d.cd;
}

// Pseudopotential, Eq. 13 with c = 1 and c_s^2 = 1/3, of a site whose shifted
// populations sum to dm (rho = rho_ref + dm).  With EOS64, a site whose density
// lies in the instance's widened spinodal interval (mix_lo < dm < mix_hi) forms
// rho and evaluates the pressure and the root in binary64; every other site
// takes the working precision.  The choice is per lane.
template <typename T, bool EOS64>
__device__ __forceinline__ T pseudopotential(T dm, const InstDev &d)
{
#pragma clang fp contract(off)
    if (EOS64 && dm > (T)d.mix_lo && dm < (T)d.mix_hi) {
        const double r = d.rho_ref + (double)dm;
        const double p = eos_pressure<double>(r, d.RT, d.a, d.b4);
        return (T)sqrt(fma(r, -1.0 / 3.0, p) * d.two_over_G);
    }
    const Consts<T> &c = consts<T>(d);
    const T rho = c.rho_ref + dm;
    const T p = eos_pressure<T>(rho, c.RT, c.a, c.b4);
    return root(fma(rho, T(-1.0 / 3.0), p) * c.two_over_G);
}

// Order-preserving map of a binary64 value onto an unsigned 64-bit key.
__device__ __forceinline__ unsigned long long order_key(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

template <typename T>
__device__ __forceinline__ bool finite_value(T v)
{
    return isfinite(v);
}

// ---------------------------------------------------------------------------
// psi pass
// ---------------------------------------------------------------------------
template <typename T, bool EOS64, int RY>
__global__ __launch_bounds__(BLOCK) void psi_pass_kernel(const InstDev *__restrict__ insts,
                                                         const Tile *__restrict__ tiles, int ntiles,
                                                         int s)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    if (s >= d.n_chunk) return;
    const gptr<const char> f = global_ptr<const char>(d.f[src_buffer(d, s)]);
    const gptr<char> psi = global_ptr<char>(d.psi);
    const unsigned long long PB = (unsigned long long)d.plane * sizeof(T);
    const unsigned long long RB = (unsigned long long)d.pitch * sizeof(T);
    const int lx = threadIdx.x & (TILE_X - 1);
    const int g = wave_index();
    const int x = tl.x0 + lx;
    const unsigned xo = (unsigned)x * sizeof(T);
    const bool track = s >= 0 && d.walls && (tl.y0 == 0 || tl.y0 + ROW_GROUPS * RY >= d.ny);
    bool bad = false;
    double wmax = -INFINITY;

    T dm[RY];                                   // rho - rho_ref per row
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = tl.y0 + g * RY + r;
        dm[r] = T(0);
        if (x < d.nx && y < d.ny) {
            const gptr<const char> rb = f + (unsigned long long)y * RB;
            T v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = ld<T>(rb + a * PB, xo);
            dm[r] = density<T>(v);
        }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = tl.y0 + g * RY + r;
        if (x < d.nx && y < d.ny) {
            const T ps = pseudopotential<T, EOS64>(dm[r], d);
            st<T>(psi + (unsigned long long)y * RB, xo, ps);
            bad |= !finite_value(ps);
            if (track && (y == 0 || y == d.ny - 1))
                wmax = fmax(wmax, eos_pressure<double>(d.rho_ref + (double)dm[r], d.RT, d.a, d.b4));
        }
    }
    if (bad) d.flag[0] = 1;
    if (track) {
        __shared__ double red[BLOCK];
        red[threadIdx.x] = wmax;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0 && red[0] > -INFINITY)
            atomicMax(&d.wall_keys[s], order_key(red[0]));
    }
}

// ---------------------------------------------------------------------------
// collision of one site (Eqs. 6, 4, 14, 3 and f* = M^-1 m*)
// ---------------------------------------------------------------------------
// f: shifted post-streaming populations g_a = f_a - w_a rho_ref of the site
// (in), shifted post-collision populations (out).  psi_c: psi at the site;
// Fx, Fy: force of Eq. 7.  The moments of g differ from those of f only in the
// mass, e and zeta rows, by rho_ref (1, -2, 1) (the rest equilibrium's
// moments), so every relaxation below is the one of Eq. 3 with those three
// rows and their equilibria shifted alike.
//
// The update is formed as an increment, f*_a = f_a + (M^-1 (m* - m))_a, not
// as M^-1 m* rebuilt from the full moments: the same quantity, but only the
// change is rounded before it is added.  A site at rest in equilibrium then
// keeps its populations bit for bit, and a nearly uniform region (the
// vapour) does not pick up the same rounding of its full populations at
// every site and every step, which in binary32 shifts the mass of a
// stationary bubble or slab by about 1e-5 over 40,000 steps.
//
// Mass of a binary32 site: rounding each of the nine stored populations
// changes the site's mass by up to half a unit in the last place of each,
// and in a stationary region the same sites round the same way at every
// step, so the error grows linearly with the step count (a flat slab, the
// same in every column, loses or gains mass coherently over all of them).
// In binary32 the rest population is therefore not formed from its
// increment: it is the site's pre-collision mass minus the eight stored
// moving populations, and that sum is rounded to binary32 up or down at
// random with the probabilities that make the stored value exact on average
// (stochastic rounding, lbm_rounding.h; `key` is the site's random word for
// this step).  Each site then keeps its mass up to one unbiased rounding of
// one population, which averages out over sites and steps instead of adding
// up.  Binary64 storage keeps the increment form.
template <typename T>
__device__ __forceinline__ void collide_site(T f[9], T psi_c, T Fx, T Fy, const Consts<T> &R,
                                             unsigned key)
{
#pragma clang fp contract(off)
    const T dm = density<T>(f);                 // rho - rho_ref
    const T rho = R.rho_ref + dm;
    const T jx = momentum_x<T>(f);
    const T jy = momentum_y<T>(f);
    const T inv_rho = recip(rho);
    // Eq. 6 with delta_t = 1
    const T vx = fma(T(0.5), Fx, jx) * inv_rho;
    const T vy = fma(T(0.5), Fy, jy) * inv_rho;
    const T v2 = fma(vx, vx, vy * vy);

    // non-conserved moments m = M f
    // (each sum a mirror-symmetric tree, as in density(); the factors 2 and 4
    // are exact, so fusing them would not change a result)
    const T axis = (f[1] + f[3]) + (f[2] + f[4]);
    const T diag = (f[5] + f[7]) + (f[6] + f[8]);
    const T m1 = fma(T(2), diag, fma(T(-4), f[0], -axis));
    const T m2 = fma(T(-2), axis, T(4) * f[0]) + diag;
    const T m4 = fma(T(2), f[3] - f[1], (f[5] + f[8]) - (f[6] + f[7]));
    const T m6 = fma(T(2), f[4] - f[2], (f[5] + f[6]) - (f[7] + f[8]));
    const T m7 = (f[1] + f[3]) - (f[2] + f[4]);
    const T m8 = (f[5] - f[6]) + (f[7] - f[8]);

    // equilibria, Eq. 4 (e and zeta rows shifted by 2 rho_ref and -rho_ref,
    // like m1 and m2: rho (-2 + 3 v^2) + 2 rho_ref, rho (1 - 3 v^2) - rho_ref)
    const T r3 = T(3) * rho;
    const T e1 = fma(r3, v2, T(-2) * dm);
    const T e2 = fma(-r3, v2, dm);
    const T rvx = rho * vx, rvy = rho * vy;   // e4 = -rvx, e6 = -rvy
    const T e7 = rho * fma(vx, vx, -(vy * vy));
    const T e8 = rvx * vy;

    // Relaxation, Eq. 3, with the source (I - Lambda/2) S of Eq. 14 and the
    // scale of the inverse transform folded into per-instance constants:
    // d_k = c_k (m*_k - m_k) = s_k c_k (m_eq_k - m_k) + c_k (1 - s_k/2) S_k.
    // For the e and zeta rows (1 - s/2) / (tau - 1/2) = s, so Li's term enters
    // as s 0.75 eps |F|^2 / psi^2.  rho and j are collision invariants up to
    // the source: m0* - m0 = 0, m3* - m3 = Fx, m5* - m5 = Fy for any s_rho,
    // s_j.
    const T vF = fma(vx, Fx, vy * Fy);
    const T li = fma(Fx, Fx, Fy * Fy) * recip(psi_c * psi_c);
    const T d1 = fma(R.e_li, li, fma(R.e_vf, vF, R.e_eq * (e1 - m1)));
    const T d2 = fma(R.z_li, li, fma(R.z_vf, vF, R.z_eq * (e2 - m2)));
    const T d4 = fma(R.q_f, Fx, -(R.q_eq * (m4 + rvx)));
    const T d6 = fma(R.q_f, Fy, -(R.q_eq * (m6 + rvy)));
    const T d7 = fma(R.n_xx, fma(vx, Fx, -(vy * Fy)), R.n_eq * (e7 - m7));
    const T d8 = fma(R.n_xy, fma(vx, Fy, vy * Fx), R.n_eq * (e8 - m8));

    // f* - f = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) (m* - m).
    // The momentum increments are divided, not multiplied by a rounded
    // reciprocal: sum_a e_a (f*_a - f_a) = 6 (d3, d5), so a reciprocal rounded
    // low (or high) would shrink (or grow) every force's momentum by the same
    // relative amount at every step.  A correctly rounded quotient (div6) has
    // no such bias.  The other moments relax, so a bias there does not
    // accumulate.
    const T d3 = div6(Fx);
    const T d5 = div6(Fy);

    const T ax = fma(T(-2), d2, -d1);       // common part of the axis increments
    const T dg = fma(T(2), d1, d2);         // common part of the diagonal ones
    const T px = fma(T(-2), d4, d3);
    const T py = fma(T(-2), d6, d5);
    const T qx = d3 + d4;
    const T qy = d5 + d6;
    T in[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) in[a] = f[a];
    f[1] += ax + px + d7;
    f[2] += ax + py - d7;
    f[3] += ax - px + d7;
    f[4] += ax - py - d7;
    f[5] += dg + qx + qy + d8;
    f[6] += dg - qx + qy - d8;
    f[7] += dg - qx - qy + d8;
    f[8] += dg + qx - qy - d8;
    if constexpr (sizeof(T) == 4) {
        // f*_0 = f_0 + sum_a (f_a - f*_a): the increment 4 (d2 - d1) plus
        // every rounding of the eight stores.  Each difference is exact while
        // the increment is below its population (Dekker) and otherwise both are
        // tiny; the sum of these small numbers rounds far below the rest
        // population's last place.  The tree is density()'s.
        T o[9];
#pragma unroll
        for (int a = 1; a < 9; ++a) o[a] = in[a] - f[a];
        const T moved = ((o[1] + o[3]) + (o[2] + o[4])) + ((o[5] + o[7]) + (o[6] + o[8]));
        f[0] = stochastic_sum(f[0], moved, key);
    } else {
        f[0] = fma(T(4), d2 - d1, f[0]);
    }
}

// Eq. 7 at the site in column l of the centre row rC, with the rows below (rS)
// and above (rN): F = -G psi(x) sum_a w_a psi(x + e_a) e_a, w = 1/3 on the
// axes and 1/12 on the diagonals.
template <typename T>
__device__ __forceinline__ void interaction_force(const T *rS, const T *rC, const T *rN, int l, T mG,
                                                  T &pc, T &Fx, T &Fy)
{
#pragma clang fp contract(off)
    pc = rC[l];
    const T pE = rC[l + 1], pW = rC[l - 1], pN = rN[l], pS = rS[l];
    const T pNE = rN[l + 1], pNW = rN[l - 1], pSW = rS[l - 1], pSE = rS[l + 1];
    const T gx = fma(T(1.0 / 12.0), (pNE - pNW) + (pSE - pSW), T(1.0 / 3.0) * (pE - pW));
    const T gy = fma(T(1.0 / 12.0), (pNE + pNW) - (pSE + pSW), T(1.0 / 3.0) * (pN - pS));
    Fx = mG * pc * gx;
    Fy = mG * pc * gy;
}

// Eq. 5: pushes the post-collision populations v of site (x, y) to x + e_a in
// fo; x wraps (xe, xw are the wrapped east and west columns); in y the
// neighbour wraps, or, through a wall, the population returns to (x, y) as
// the opposite one (halfway bounce-back).
template <typename T, bool WT = false>
__device__ __forceinline__ void push_store(gptr<char> fo, unsigned long long PB, const T v[9], unsigned xo,
                                           unsigned xeo, unsigned xwo, int y, int ny,
                                           unsigned long long row_bytes, int walls)
{
    const bool top = (y == ny - 1), bot = (y == 0);
    int yn = y + 1, ys = y - 1;
    if (!walls) {
        if (top) yn = 0;
        if (bot) ys = ny - 1;
    }
    const gptr<char> rc = fo + (unsigned long long)y * row_bytes;
    const gptr<char> rn = fo + (unsigned long long)yn * row_bytes;
    const gptr<char> rs = fo + (unsigned long long)ys * row_bytes;
    stw<T, WT>(rc, xo, v[0]);
    stw<T, WT>(rc + 1 * PB, xeo, v[1]);
    stw<T, WT>(rc + 3 * PB, xwo, v[3]);
    if (walls && top) {
        stw<T, WT>(rc + 4 * PB, xo, v[2]);
        stw<T, WT>(rc + 7 * PB, xo, v[5]);
        stw<T, WT>(rc + 8 * PB, xo, v[6]);
    } else {
        stw<T, WT>(rn + 2 * PB, xo, v[2]);
        stw<T, WT>(rn + 5 * PB, xeo, v[5]);
        stw<T, WT>(rn + 6 * PB, xwo, v[6]);
    }
    if (walls && bot) {
        stw<T, WT>(rc + 2 * PB, xo, v[4]);
        stw<T, WT>(rc + 5 * PB, xo, v[7]);
        stw<T, WT>(rc + 6 * PB, xo, v[8]);
    } else {
        stw<T, WT>(rs + 4 * PB, xo, v[4]);
        stw<T, WT>(rs + 7 * PB, xwo, v[7]);
        stw<T, WT>(rs + 8 * PB, xeo, v[8]);
    }
}

// ---------------------------------------------------------------------------
// force + collide + stream pass
// ---------------------------------------------------------------------------
template <typename T, int RY>
__global__ __launch_bounds__(BLOCK) void collide_stream_kernel(const InstDev *__restrict__ insts,
                                                               const Tile *__restrict__ tiles,
                                                               int ntiles, int s)
{
    constexpr int TY = ROW_GROUPS * RY;
    constexpr int LW = TILE_X + 2;
    __shared__ T sp[(TY + 2) * LW];

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    if (s >= d.n_chunk) return;
    const int sb = src_buffer(d, s);
    const gptr<const char> f = global_ptr<const char>(d.f[sb]);
    const gptr<char> fo = global_ptr<char>(d.f[sb ^ 1]);
    const gptr<const char> psi = global_ptr<const char>(d.psi);
    const unsigned long long PB = (unsigned long long)d.plane * sizeof(T);
    const unsigned long long RB = (unsigned long long)d.pitch * sizeof(T);
    const int nx = d.nx, ny = d.ny;
    const unsigned sw = hash32((unsigned)(d.step + s));

    // psi of the tile and a one-site ring; x wraps, y wraps or mirrors at walls
    for (int k = threadIdx.x; k < (TY + 2) * LW; k += BLOCK) {
        const int ly = k / LW;
        const int lxx = k - ly * LW;
        int gx = (tl.x0 - 1 + lxx) % nx;
        if (gx < 0) gx += nx;
        int gy = tl.y0 - 1 + ly;
        if (d.walls) {
            gy = gy < 0 ? 0 : (gy > ny - 1 ? ny - 1 : gy);
        } else {
            gy %= ny;
            if (gy < 0) gy += ny;
        }
        sp[k] = ld_lane<T>(psi, (unsigned long long)gy * RB + (unsigned)gx * sizeof(T));
    }
    __syncthreads();

    const Consts<T> &R = consts<T>(d);
    const int lx = threadIdx.x & (TILE_X - 1);
    const int g = wave_index();
    const int x = tl.x0 + lx;
    if (x >= nx) return;
    const unsigned xo = (unsigned)x * sizeof(T);
    const unsigned xeo = (unsigned)((x + 1 == nx) ? 0 : x + 1) * sizeof(T);
    const unsigned xwo = (unsigned)((x == 0) ? nx - 1 : x - 1) * sizeof(T);
    const unsigned cw = column_word(x, nx);

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int ly = g * RY + r;
        const int y = tl.y0 + ly;
        if (y >= ny) break;
        const gptr<const char> rb = f + (unsigned long long)y * RB;
        T v[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) v[a] = ld<T>(rb + a * PB, xo);

        T pc, Fx, Fy;
        interaction_force<T>(sp + ly * LW, sp + (ly + 1) * LW, sp + (ly + 2) * LW, lx + 1, R.mG, pc,
                             Fx, Fy);
        collide_site<T>(v, pc, Fx, Fy, R, cw ^ row_word(y, ny, sw));
        push_store<T>(fo, PB, v, xo, xeo, xwo, y, ny, RB, d.walls);
    }
}

// ---------------------------------------------------------------------------
// fused pass: the whole step in one kernel
// ---------------------------------------------------------------------------
// A block owns a strip of TILE_X columns and H rows.  Its four wavefronts walk
// down the strip together, wavefront w taking rows y0 - 1 + 4k + w at
// iteration k: each forms rho and psi (Eqs. 15, 13) of its row from the nine
// populations loaded during the previous iteration and writes psi into a
// 16-row ring in LDS.  The row it handled two iterations earlier then has psi
// above and below it in the ring, and is collided from the populations kept
// in registers (Eqs. 7, 6, 4, 14, 3) and pushed to the other buffer (Eq. 5).
// Every population is read from memory once per step (the one-row and
// one-column rings are re-read by the neighbouring strips), and psi never
// leaves LDS.
//
// The loads of a row are issued one iteration before the row is used, so each
// wavefront keeps the next row's loads in flight while it works; the
// collision's stores and the barrier do not wait behind them.  psi of the row
// handled now is formed before the collision, so that the loads it waits for
// are the last ones issued before the prefetch.  The two ring columns left and
// right of the strip are loaded one population per lane (lanes 0-8 and 16-24;
// the other lanes load a copy that is not used) and summed across lanes into
// lanes 1 and 17.
//
// Ring hazards: in iteration k the block writes psi of rows y0-1+4k .. y0+2+4k
// and reads rows y0+4k-10 .. y0+4k-5, all written before the previous
// barrier; the two sets are 4 to 12 rows apart, so with 16 slots no slot is
// written while another wavefront reads it, and one barrier per iteration
// suffices.

// The value of lane i + N of the same 16-lane row (a DPP row shift, a plain
// register move: no LDS, no address arithmetic); lanes whose source lies
// outside the row get 0.
template <int N>
__device__ __forceinline__ float row_next(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x100 + N, 0xF, 0xF, true));
}

template <int N>
__device__ __forceinline__ double row_next(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x100 + N, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x100 + N, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The value of lane i - N of the same 16-lane row (a DPP row shift the other
// way); lanes whose source lies outside the row get 0.
template <int N>
__device__ __forceinline__ float row_prev(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + N, 0xF, 0xF, true));
}

template <int N>
__device__ __forceinline__ double row_prev(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x110 + N, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x110 + N, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Lanes b .. b+8 (b = 0 or 16) hold populations 0..8 of one ring column;
// returns in lane b + 1 the column's rho - rho_ref, summed in the order of
// density().  Every lane of the wavefront must call it.
template <typename T>
__device__ __forceinline__ T halo_density(T v)
{
    const T s1 = v + row_next<2>(v);          // lanes b+1, b+2, b+5, b+6: v1+v3, v2+v4, v5+v7, v6+v8
    const T s2 = s1 + row_next<1>(s1);        // lanes b+1, b+5: the axis and the diagonal sums
    const T s3 = s2 + row_next<4>(s2);        // lane b+1: the eight moving populations
    return s3 + row_prev<1>(v);               // lane b+1: plus v0 from lane b
}

// Memory row of lattice row l (ghost rows -1 and ny mirror at walls, wrap
// otherwise).
__device__ __forceinline__ int memory_row(int l, int ny, int walls)
{
    if (walls) return l < 0 ? 0 : (l > ny - 1 ? ny - 1 : l);
    return l < 0 ? l + ny : (l >= ny ? l - ny : l);
}

template <typename T, bool EOS64, int H>
__global__ __launch_bounds__(BLOCK) void fused_kernel(const InstDev *__restrict__ insts,
                                                      const Tile *__restrict__ tiles, int ntiles, int s,
                                                      int alternate, int write_through)
{
    constexpr int RING = 16;
    constexpr int LW = TILE_X + 2;
    constexpr int NLOAD = (H + 2 + ROW_GROUPS - 1) / ROW_GROUPS;
    constexpr int NK = NLOAD + 2;
    static_assert(H % ROW_GROUPS == 0, "strip height must be a multiple of the row groups");
    __shared__ T ring[RING * LW];

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    if (s >= d.n_chunk) return;
    const int sb = src_buffer(d, s);
    const gptr<const char> f = global_ptr<const char>(d.f[sb]);
    const gptr<char> fo = global_ptr<char>(d.f[sb ^ 1]);
    const unsigned long long PB = (unsigned long long)d.plane * sizeof(T);
    const unsigned long long RB = (unsigned long long)d.pitch * sizeof(T);
    const int nx = d.nx, ny = d.ny, walls = d.walls;
    const int lane = threadIdx.x & (TILE_X - 1);
    const int w = wave_index();
    const int x = tl.x0 + lane;
    const int xl = x < nx ? x : x % nx;                       // column this lane loads
    const unsigned sw = hash32((unsigned)(d.step + s));
    const unsigned cw = column_word(x, nx);
    const unsigned xo = (unsigned)x * sizeof(T), xlo = (unsigned)xl * sizeof(T);
    const unsigned xeo = (unsigned)((x + 1 >= nx) ? 0 : x + 1) * sizeof(T);
    const unsigned xwo = (unsigned)((x == 0) ? nx - 1 : x - 1) * sizeof(T);
    // ring columns: lane 16 c + a (a < 9) loads population a of column c
    const int hp = lane & 15;
    const bool hlane = lane < 32 && hp < 9;
    const int hcol = lane < 16 ? (tl.x0 == 0 ? nx - 1 : tl.x0 - 1) : (tl.x0 + TILE_X) % nx;
    const unsigned long long hoff = (unsigned long long)(hlane ? hp : 0) * PB + (unsigned)hcol * sizeof(T);
    const bool hroot = lane == 1 || lane == 17;
    const int hslot = lane == 1 ? 0 : LW - 1;
    const int y_end = min(tl.y0 + H, ny);                     // rows collided: [y0, y_end)
    const bool track = walls && (tl.y0 == 0 || tl.y0 + H >= ny);
    const Consts<T> &R = consts<T>(d);
    const T mG = R.mG;

    bool bad = false;
    double wmax = -INFINITY;
    // rows of iterations k + 1 (fq), k (fn), k - 1 (fa) and k - 2 (fb); hq, hn:
    // ring column populations of rows k + 1 and k
    T fq[9], fn[9], fa[9], fb[9], hq = T(0), hn = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) fq[a] = fn[a] = fa[a] = fb[a] = T(0);

    // The tile's rows y0 - 1 .. l_last are walked upwards.  When the whole
    // grid is resident at once (`alternate`), every other band of tiles (odd
    // y0 / H) walks downwards instead: two vertically neighbouring tiles,
    // which then run side by side, reach the rows around their common edge
    // at about the same time (both at the start or both at the end of their
    // walks), so the second reader of those rows finds them in L2, where
    // upward walks would read them a whole walk apart.  A grid that runs in
    // successive waves of blocks keeps the upward walk: there a band's
    // blocks start about when the band below them finishes, which lines up
    // their common rows already.
    const int l_first = tl.y0 - 1;
    const int l_last = min(tl.y0 + H, ny);
    const bool down = alternate && ((tl.y0 / H) & 1) != 0;
    const int dir = down ? -1 : 1;
    const int l_start = down ? l_last : l_first;
    auto row_of = [&](int k) { return l_start + dir * (ROW_GROUPS * k + w); };

    // Every load is issued unconditionally, so that the loads in flight are
    // the same on every path and the compiler's wait counts stay exact (a
    // load under a branch makes it wait for all outstanding loads, the
    // prefetch included).  Rows past the walk's last row are clamped to that
    // row (already being loaded by another wavefront of the block, so served
    // from cache) and never used.
    auto row_loaded = [&](int k, int l) { return k < NLOAD && l >= l_first && l <= l_last; };
    auto load_row = [&](int k, T v[9], T &h) {
        const int l = min(max(row_of(k), l_first), l_last);
        const gptr<const char> rb = f + (unsigned long long)memory_row(l, ny, walls) * RB;
        h = ld_lane<T>(rb, hoff);
#pragma unroll
        for (int a = 0; a < 9; ++a) v[a] = ld<T>(rb + a * PB, xlo);
    };
    load_row(0, fn, hn);

    // Iteration k: loads row k + 1 (when `next`), forms psi of row k and
    // collides row k - 2 (rows counted along the walk).
    auto iteration = [&](int k, bool next) __attribute__((always_inline)) {
        const int l = row_of(k);                              // row handled now
        const bool have = row_loaded(k, l);
        if (next) load_row(k + 1, fq, hq);                    // in flight until the next iteration

        T *row = ring + (l & (RING - 1)) * LW;
        if (have) {
            const T dm_h = halo_density<T>(hn);
            if (hroot) {
                const T ph = pseudopotential<T, EOS64>(dm_h, d);
                row[hslot] = ph;
                bad |= !finite_value(ph);
            }
        }

        // psi of the row handled now
        if (have) {
            const T dm = density<T>(fn);
            const T ps = pseudopotential<T, EOS64>(dm, d);
            row[lane + 1] = ps;
            bad |= !finite_value(ps);
            if (track && (l == 0 || l == ny - 1) && l >= tl.y0 && l < y_end && x < nx)
                wmax = fmax(wmax, eos_pressure<double>(d.rho_ref + (double)dm, d.RT, d.a, d.b4));
        }
        // collide the row handled two iterations ago; its psi neighbours
        // were handled before the last barrier, and this iteration's psi
        // rows lie 4 to 12 rows from them, so they never share a ring slot
        const int c = l - dir * 2 * ROW_GROUPS;
        if (k >= 2 && c >= tl.y0 && c < y_end && x < nx) {
            const T *rS = ring + ((c - 1) & (RING - 1)) * LW;
            const T *rC = ring + (c & (RING - 1)) * LW;
            const T *rN = ring + ((c + 1) & (RING - 1)) * LW;
            T pc, Fx, Fy;
            interaction_force<T>(rS, rC, rN, lane + 1, mG, pc, Fx, Fy);
            collide_site<T>(fb, pc, Fx, Fy, R, cw ^ row_word(c, ny, sw));
            // write-through stores leave no dirty lines in L2 for the
            // kernel's end to write back (chosen per batch, uniform)
            if (write_through) push_store<T, true>(fo, PB, fb, xo, xeo, xwo, c, ny, RB, walls);
            else push_store<T, false>(fo, PB, fb, xo, xeo, xwo, c, ny, RB, walls);
        }

        __syncthreads();
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            fb[a] = fa[a];
            fa[a] = fn[a];
            if (next) fn[a] = fq[a];
        }
        if (next) hn = hq;
    };

    // Unrolled by four so that the rotation of the four row buffers
    // (next -> now -> one ago -> two ago) becomes register renaming; the last
    // three iterations load nothing.
#pragma unroll 4
    for (int k = 0; k < NLOAD - 1; ++k) iteration(k, true);
#pragma unroll
    for (int k = NLOAD - 1; k < NK; ++k) iteration(k, false);
    if (bad) d.flag[0] = 1;
    if (track) {
        __shared__ double red[BLOCK];
        red[threadIdx.x] = wmax;
        __syncthreads();
        for (int k2 = BLOCK / 2; k2 > 0; k2 >>= 1) {
            if (threadIdx.x < k2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k2]);
            __syncthreads();
        }
        if (threadIdx.x == 0 && red[0] > -INFINITY) atomicMax(&d.wall_keys[s], order_key(red[0]));
    }
}


// ---------------------------------------------------------------------------
// paired fused pass: the fused pass with two neighbouring sites per lane
// ---------------------------------------------------------------------------
// Same walk as fused_kernel over strips of 2 * TILE_X columns; lane l owns the
// columns x0 + 2l and x0 + 2l + 1 and moves both with one two-element access
// per population plane (a 64-wide wavefront reads 512 B of a plane at once),
// which the memory system serves markedly faster than one element per lane.
// Populations moving in x land on the neighbouring pair: the value entering a
// pair from the left comes from the lane to the left (a lane shuffle), so every
// store stays aligned; the one value that crosses a strip edge is stored on
// its own by the edge lane.  nx must be even, so that a pair never straddles
// the end of a row (the host enforces it).
typedef float float_pair __attribute__((ext_vector_type(2)));
typedef double double_pair __attribute__((ext_vector_type(2)));

template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using type = float_pair;
};
template <>
struct Pair<double> {
    using type = double_pair;
};

template <typename T>
__device__ __forceinline__ typename Pair<T>::type ldp(gptr<const char> row_base, unsigned lane_off)
{
    return *(gptr<const typename Pair<T>::type>)(scalar_base(row_base) + lane_offset(lane_off));
}

template <typename T>
__device__ __forceinline__ void stp(gptr<char> row_base, unsigned lane_off, T a, T b)
{
    typename Pair<T>::type v;
    v.x = a;
    v.y = b;
    *(gptr<typename Pair<T>::type>)(scalar_base(row_base) + lane_offset(lane_off)) = v;
}

// Lane-position facts of a pair (all offsets in bytes).
struct PairLane {
    unsigned xo;        // the pair's own first column
    unsigned xo1;       // the pair's second column
    unsigned east_ovf;  // where the last pair's right value goes moving east
    unsigned west_ovf;  // where lane 0's left value goes moving west
    bool valid;         // the pair holds lattice sites
    bool first;         // lane 0
    bool last;          // the strip's last valid pair
};

// Stores one direction's post-collision pair (v0 at column cx, v1 at cx + 1)
// into `row`, shifted in x by shift = 0, +1 (east) or -1 (west).  All lanes
// must call it together (it shuffles).
template <typename T>
__device__ __forceinline__ void store_pair(gptr<char> row, int shift, T v0, T v1, const PairLane &pl)
{
    if (shift == 0) {
        if (pl.valid) stp<T>(row, pl.xo, v0, v1);
    } else if (shift > 0) {
        const T up = __shfl_up(v1, 1);            // right value of the pair to the left
        if (pl.valid) {
            if (pl.first) st<T>(row, pl.xo1, v0);
            else stp<T>(row, pl.xo, up, v0);
            if (pl.last) st<T>(row, pl.east_ovf, v1);
        }
    } else {
        const T dn = __shfl_down(v0, 1);          // left value of the pair to the right
        if (pl.valid) {
            if (pl.last) st<T>(row, pl.xo, v1);
            else stp<T>(row, pl.xo, v1, dn);
            if (pl.first) st<T>(row, pl.west_ovf, v0);
        }
    }
}

template <typename T, bool EOS64, int H>
__global__ __launch_bounds__(BLOCK) void fused2_kernel(const InstDev *__restrict__ insts,
                                                       const Tile *__restrict__ tiles, int ntiles, int s,
                                                       int alternate)
{
    using V = typename Pair<T>::type;
    constexpr int RING = 16;
    constexpr int SW = 2 * TILE_X;
    constexpr int LW = SW + 2;
    constexpr int NLOAD = (H + 2 + ROW_GROUPS - 1) / ROW_GROUPS;
    constexpr int NK = NLOAD + 2;
    static_assert(H % ROW_GROUPS == 0, "strip height must be a multiple of the row groups");
    __shared__ T ring[RING * LW];

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    if (s >= d.n_chunk) return;
    const int sb = src_buffer(d, s);
    const gptr<const char> f = global_ptr<const char>(d.f[sb]);
    const gptr<char> fo = global_ptr<char>(d.f[sb ^ 1]);
    const unsigned long long PB = (unsigned long long)d.plane * sizeof(T);
    const unsigned long long RB = (unsigned long long)d.pitch * sizeof(T);
    const int nx = d.nx, ny = d.ny, walls = d.walls;
    const int lane = threadIdx.x & (TILE_X - 1);
    const int w = wave_index();
    const int cx = tl.x0 + 2 * lane;                         // the pair's first column
    const unsigned sw = hash32((unsigned)(d.step + s));
    const unsigned cw0 = column_word(cx, nx), cw1 = column_word(cx + 1, nx);
    const int last_cx = min(tl.x0 + SW, nx) - 2;
    PairLane pl;
    pl.valid = cx < nx;
    pl.first = lane == 0;
    pl.last = cx == last_cx;
    pl.xo = (unsigned)cx * sizeof(T);
    pl.xo1 = (unsigned)(cx + 1) * sizeof(T);
    pl.east_ovf = (unsigned)((cx + 2) % nx) * sizeof(T);
    pl.west_ovf = (unsigned)(tl.x0 == 0 ? nx - 1 : tl.x0 - 1) * sizeof(T);
    const unsigned xlo = (unsigned)(pl.valid ? cx : cx % nx) * sizeof(T);   // pair loaded (wrapped)
    // ring columns: lane 16 c + a (a < 9) loads population a of column c
    const int hp = lane & 15;
    const bool hlane = lane < 32 && hp < 9;
    const int hcol = lane < 16 ? (tl.x0 == 0 ? nx - 1 : tl.x0 - 1) : (tl.x0 + SW) % nx;
    const unsigned long long hoff = (unsigned long long)(hlane ? hp : 0) * PB + (unsigned)hcol * sizeof(T);
    const bool hroot = lane == 1 || lane == 17;
    const int hslot = lane == 1 ? 0 : LW - 1;
    const int y_end = min(tl.y0 + H, ny);
    const bool track = walls && (tl.y0 == 0 || tl.y0 + H >= ny);
    const Consts<T> &R = consts<T>(d);
    const T mG = R.mG;

    bool bad = false;
    double wmax = -INFINITY;
    V fn[9], fa[9], fb[9];
    T hn = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        fn[a].x = fn[a].y = T(0);
        fa[a].x = fa[a].y = T(0);
        fb[a].x = fb[a].y = T(0);
    }

    // Unlike fused_kernel, the loads stay under their row conditions and the
    // ring-column load under its lane mask.  The compiler then waits for the
    // prefetched row during the collision, but this kernel is bound by memory
    // bandwidth at four wavefronts per SIMD, and the unconditional form
    // (more load instructions, the next row's loads overlapping the stores)
    // measured 3 % slower on the 8192 x 4096 grid.
    // Rows y0 - 1 .. l_last, walked upwards or, with `alternate`, downwards
    // in every other band of tiles, as in fused_kernel.
    const int l_first = tl.y0 - 1;
    const int l_last = min(tl.y0 + H, ny);
    const bool down = alternate && ((tl.y0 / H) & 1) != 0;
    const int dir = down ? -1 : 1;
    const int l_start = down ? l_last : l_first;
    auto row_of = [&](int k) { return l_start + dir * (ROW_GROUPS * k + w); };
    auto row_loaded = [&](int k, int l) { return k < NLOAD && l >= l_first && l <= l_last; };
    auto load_row = [&](int k, V v[9], T &h) {
        const int l = row_of(k);
        if (row_loaded(k, l)) {
            const gptr<const char> rb = f + (unsigned long long)memory_row(l, ny, walls) * RB;
            if (hlane) h = ld_lane<T>(rb, hoff);
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = ldp<T>(rb + a * PB, xlo);
        }
    };
    load_row(0, fn, hn);

#pragma unroll 4
    for (int k = 0; k < NK; ++k) {
        const int l = row_of(k);
        const bool have = row_loaded(k, l);
        V fq[9];
        T hq = T(0);
#pragma unroll
        for (int a = 0; a < 9; ++a) fq[a].x = fq[a].y = T(0);
        load_row(k + 1, fq, hq);

        T *row = ring + (l & (RING - 1)) * LW;
        if (have) {
            const T dm_h = halo_density<T>(hn);
            if (hroot) {
                const T ph = pseudopotential<T, EOS64>(dm_h, d);
                row[hslot] = ph;
                bad |= !finite_value(ph);
            }
        }

        // collide and push the row handled two iterations ago
        const int c = l - dir * 2 * ROW_GROUPS;
        if (k >= 2 && c >= tl.y0 && c < y_end) {
            const T *rS = ring + ((c - 1) & (RING - 1)) * LW;
            const T *rC = ring + (c & (RING - 1)) * LW;
            const T *rN = ring + ((c + 1) & (RING - 1)) * LW;
            T v0[9], v1[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                v0[a] = fb[a].x;
                v1[a] = fb[a].y;
            }
            T pc, Fx, Fy;
            interaction_force<T>(rS, rC, rN, 2 * lane + 1, mG, pc, Fx, Fy);
            const unsigned rw = row_word(c, ny, sw);
            collide_site<T>(v0, pc, Fx, Fy, R, cw0 ^ rw);
            interaction_force<T>(rS, rC, rN, 2 * lane + 2, mG, pc, Fx, Fy);
            collide_site<T>(v1, pc, Fx, Fy, R, cw1 ^ rw);

            // Eq. 5 with halfway bounce-back; the row conditions are uniform
            const bool top = (c == ny - 1), bot = (c == 0);
            int yn = c + 1, ys = c - 1;
            if (!walls) {
                if (top) yn = 0;
                if (bot) ys = ny - 1;
            }
            const gptr<char> r0 = fo + (unsigned long long)c * RB;
            const gptr<char> rn = fo + (unsigned long long)yn * RB;
            const gptr<char> rs = fo + (unsigned long long)ys * RB;
            store_pair<T>(r0, 0, v0[0], v1[0], pl);
            store_pair<T>(r0 + 1 * PB, +1, v0[1], v1[1], pl);
            store_pair<T>(r0 + 3 * PB, -1, v0[3], v1[3], pl);
            if (walls && top) {
                store_pair<T>(r0 + 4 * PB, 0, v0[2], v1[2], pl);
                store_pair<T>(r0 + 7 * PB, 0, v0[5], v1[5], pl);
                store_pair<T>(r0 + 8 * PB, 0, v0[6], v1[6], pl);
            } else {
                store_pair<T>(rn + 2 * PB, 0, v0[2], v1[2], pl);
                store_pair<T>(rn + 5 * PB, +1, v0[5], v1[5], pl);
                store_pair<T>(rn + 6 * PB, -1, v0[6], v1[6], pl);
            }
            if (walls && bot) {
                store_pair<T>(r0 + 2 * PB, 0, v0[4], v1[4], pl);
                store_pair<T>(r0 + 5 * PB, 0, v0[7], v1[7], pl);
                store_pair<T>(r0 + 6 * PB, 0, v0[8], v1[8], pl);
            } else {
                store_pair<T>(rs + 4 * PB, 0, v0[4], v1[4], pl);
                store_pair<T>(rs + 7 * PB, -1, v0[7], v1[7], pl);
                store_pair<T>(rs + 8 * PB, +1, v0[8], v1[8], pl);
            }
        }

        // psi of the row handled now
        if (have) {
            T e0[9], e1[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                e0[a] = fn[a].x;
                e1[a] = fn[a].y;
            }
            const T dm0 = density<T>(e0), dm1 = density<T>(e1);
            const T p0 = pseudopotential<T, EOS64>(dm0, d);
            const T p1 = pseudopotential<T, EOS64>(dm1, d);
            row[2 * lane + 1] = p0;
            row[2 * lane + 2] = p1;
            bad |= !finite_value(p0) || !finite_value(p1);
            if (track && (l == 0 || l == ny - 1) && l >= tl.y0 && l < y_end && pl.valid) {
                wmax = fmax(wmax, eos_pressure<double>(d.rho_ref + (double)dm0, d.RT, d.a, d.b4));
                wmax = fmax(wmax, eos_pressure<double>(d.rho_ref + (double)dm1, d.RT, d.a, d.b4));
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            fb[a] = fa[a];
            fa[a] = fn[a];
            fn[a] = fq[a];
        }
        hn = hq;
    }
    if (bad) d.flag[0] = 1;
    if (track) {
        __shared__ double red[BLOCK];
        red[threadIdx.x] = wmax;
        __syncthreads();
        for (int k2 = BLOCK / 2; k2 > 0; k2 >>= 1) {
            if (threadIdx.x < k2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k2]);
            __syncthreads();
        }
        if (threadIdx.x == 0 && red[0] > -INFINITY) atomicMax(&d.wall_keys[s], order_key(red[0]));
    }
}

// ---------------------------------------------------------------------------
// two-step pass: steps t and t + 1 in one kernel
// ---------------------------------------------------------------------------
// A block owns a strip of T2_OUT = 58 output columns and H rows, and its four
// wavefronts walk it as in fused_kernel, but every lane holds one of 64
// columns that reach three sites past the strip on each side: lane l is
// column x0 - 3 + l.  Per iteration k, wavefront w:
//
//   step t      loads the populations of row y0 - 3 + 4(k + 1) + w (one
//               iteration ahead), forms rho and psi (Eqs. 15, 13) of the row
//               loaded last into a psi ring, and collides the row loaded two
//               iterations ago (Eqs. 7, 6, 4, 14, 3) in lanes 1 .. 62; the
//               post-collision populations are pushed (Eq. 5, halfway
//               bounce-back at walls) into a ring of rows in LDS instead of
//               memory;
//   step t + 1  reads a row of that ring once all three rows that push into
//               it have been collided (four iterations behind), forms rho
//               and psi of t + 1 in lanes 2 .. 61, and collides the row read
//               two iterations ago in the 58 output lanes 3 .. 60, pushing to
//               the other population buffer in memory.
//
// So each population is read from memory once and written once per two
// steps; the intermediate state never leaves LDS.  The dependence reaches
// three sites per two steps (psi of a neighbour, then streaming, twice), which
// is where the three extra columns and rows on each side go.  Each output
// site is computed with the arithmetic of fused_kernel in the same order.
//
// Ring hazards (one barrier per iteration): in iteration k the step-t
// collisions write rows y0 - 12 + 4k .. y0 - 7 + 4k of the 12-row population
// ring and the step-t + 1 reads take rows y0 - 17 + 4k .. y0 - 14 + 4k, all
// completed before the previous barrier; rows 12 apart share a slot, and
// every slot read in iteration k is next written in iteration k + 1 or
// later.  The two psi rings follow fused_kernel's pattern (rows written and
// read in one iteration 4 to 12 apart, 16 slots).
//
// A launch with index s advances every instance with s < ceil(n / 2) (n its
// steps in the chunk) by steps 2s and 2s + 1, reading buffer (cur + s) mod 2
// and writing the other; when n is odd, launch (n - 1) / 2 takes only step
// n - 1, its step-t collisions pushing to memory.  An instance's buffer
// therefore flips ceil(n / 2) times per chunk.
constexpr int T2_HALO = 3;
constexpr int T2_OUT = TILE_X - 2 * T2_HALO;
static_assert(T2_OUT == TWOSTEP_COLS, "two-step strip width");

template <typename T, bool EOS64, int H>
__global__ __launch_bounds__(BLOCK) void twostep_kernel(const InstDev *__restrict__ insts,
                                                        const Tile *__restrict__ tiles, int ntiles, int s,
                                                        int write_through)
{
    constexpr int RP = 16;
    constexpr int RF = 12;
    constexpr int NA = (H + 2 * T2_HALO + ROW_GROUPS - 1) / ROW_GROUPS;
    constexpr int NK = H / ROW_GROUPS + 7;
    static_assert(H % ROW_GROUPS == 0, "strip height must be a multiple of the row groups");
    __shared__ T psiA[RP * TILE_X];
    __shared__ T psiB[RP * TILE_X];
    __shared__ __align__(16) T f1[RF * 9 * TILE_X];
    static_assert(sizeof(f1) >= 2 * BLOCK * sizeof(double), "the wall reduction reuses the ring");

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    const int n = d.n_chunk;
    if (s >= ((n + 1) >> 1)) return;
    const bool single = (n & 1) && s == (n >> 1);          // the chunk's last, odd step alone
    const int sb = src_buffer(d, s);
    const gptr<const char> f = global_ptr<const char>(d.f[sb]);
    const gptr<char> fo = global_ptr<char>(d.f[sb ^ 1]);
    const unsigned long long PB = (unsigned long long)d.plane * sizeof(T);
    const unsigned long long RB = (unsigned long long)d.pitch * sizeof(T);
    const int nx = d.nx, ny = d.ny, walls = d.walls;
    const int lane = threadIdx.x & (TILE_X - 1);
    const int w = wave_index();
    const int X = tl.x0 - T2_HALO + lane;                   // the lane's column (unwrapped)
    int xl = X % nx;
    if (xl < 0) xl += nx;
    const unsigned xlo = (unsigned)xl * sizeof(T);
    const bool out = lane >= T2_HALO && lane < TILE_X - T2_HALO && X < nx;   // X >= x0 >= 0 here
    const unsigned xo = xlo;
    const unsigned xeo = (unsigned)((xl + 1 == nx) ? 0 : xl + 1) * sizeof(T);
    const unsigned xwo = (unsigned)((xl == 0) ? nx - 1 : xl - 1) * sizeof(T);
    const unsigned swA = hash32((unsigned)(d.step + 2 * s));      // steps t and t + 1
    const unsigned swB = hash32((unsigned)(d.step + 2 * s + 1));
    const unsigned cw = column_word(xl, nx);
    const bool lane_a = lane >= 1 && lane <= TILE_X - 2;    // step-t collisions
    const bool lane_b = lane >= 2 && lane <= TILE_X - 3;    // step-t + 1 densities
    const int y_end = min(tl.y0 + H, ny);                   // rows output: [y0, y_end)
    const int lA_first = tl.y0 - 3, lA_last = y_end + 2;    // rows loaded for step t
    const bool track = walls && (tl.y0 == 0 || tl.y0 + H >= ny);
    const Consts<T> &R = consts<T>(d);
    const T mG = R.mG;

    bool bad = false;
    double wmaxA = -INFINITY, wmaxB = -INFINITY;
    T fq[9], fn[9], fa[9], fb[9], gn[9], ga[9], gb[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fq[a] = fn[a] = fa[a] = fb[a] = gn[a] = ga[a] = gb[a] = T(0);

    auto rowA = [&](int k) { return lA_first + ROW_GROUPS * k + w; };
    auto rowB = [&](int m) { return tl.y0 - 1 + ROW_GROUPS * m + w; };
    auto f1row = [&](int r) { return f1 + ((r + RF) % RF) * (9 * TILE_X); };   // r >= -3
    // loads are issued unconditionally (rows past the last needed one are
    // clamped to it) so that the compiler's wait counts stay exact
    // returns the memory row, which is also the lattice row of a collided
    // site (the rows collided at step t lie inside the walls)
    auto load_row = [&](int k, T v[9]) {
        const int l = min(rowA(k), lA_last);
        // rows reach three past the strip, so a periodic grid of fewer than
        // three rows wraps more than once; the row is uniform over the
        // wavefront, and these loops (at most one pass on three rows or more)
        // run on the scalar unit, where a modulo would take a vector division
        int mr = l;
        if (walls) {
            mr = min(max(l, 0), ny - 1);
        } else {
            while (mr < 0) mr += ny;
            while (mr >= ny) mr -= ny;
        }
        const gptr<const char> rb = f + (unsigned long long)mr * RB;
#pragma unroll
        for (int a = 0; a < 9; ++a) v[a] = ld<T>(rb + a * PB, xlo);
        return mr;
    };
    // memory rows of fq, fn, fa, fb (uniform over the wavefront)
    int mq = 0, mn = load_row(0, fn), ma = 0, mb = 0;

    auto iteration = [&](int k, bool next) __attribute__((always_inline)) {
        if (next) mq = load_row(k + 1, fq);

        // step t: rho and psi of the row loaded last
        const int l = rowA(k);
        if (k < NA && l <= lA_last) {
            const T dm = density<T>(fn);
            const T ps = pseudopotential<T, EOS64>(dm, d);
            psiA[(l & (RP - 1)) * TILE_X + lane] = ps;
            bad |= !finite_value(ps);
            if (track && (l == 0 || l == ny - 1) && l >= tl.y0 && l < y_end && out)
                wmaxA = fmax(wmaxA, eos_pressure<double>(d.rho_ref + (double)dm, d.RT, d.a, d.b4));
        }

        // step t: collide the row loaded two iterations ago
        const int c = rowA(k - 2);
        const bool crow = k >= 2 && c >= tl.y0 - 2 && c <= y_end + 1 && (!walls || (c >= 0 && c < ny));
        if (crow && lane_a) {
            const T *rS = psiA + ((c - 1) & (RP - 1)) * TILE_X;
            const T *rC = psiA + (c & (RP - 1)) * TILE_X;
            const T *rN = psiA + ((c + 1) & (RP - 1)) * TILE_X;
            T pc, Fx, Fy;
            interaction_force<T>(rS, rC, rN, lane, mG, pc, Fx, Fy);
            // rows beyond a periodic edge are the wrapped rows' sites
            collide_site<T>(fb, pc, Fx, Fy, R, cw ^ row_word(mb, ny, swA));
            if (single) {
                // the odd last step of the chunk: straight to memory
                if (out && c >= tl.y0 && c < y_end) {
                    if (write_through) push_store<T, true>(fo, PB, fb, xo, xeo, xwo, c, ny, RB, walls);
                    else push_store<T>(fo, PB, fb, xo, xeo, xwo, c, ny, RB, walls);
                }
            } else {
                // Eq. 5 into the LDS rows of t + 1; halfway bounce-back at walls
                T *r0 = f1row(c);
                r0[0 * TILE_X + lane] = fb[0];
                r0[1 * TILE_X + lane + 1] = fb[1];
                r0[3 * TILE_X + lane - 1] = fb[3];
                if (walls && c == ny - 1) {
                    r0[4 * TILE_X + lane] = fb[2];
                    r0[7 * TILE_X + lane] = fb[5];
                    r0[8 * TILE_X + lane] = fb[6];
                } else {
                    T *rn = f1row(c + 1);
                    rn[2 * TILE_X + lane] = fb[2];
                    rn[5 * TILE_X + lane + 1] = fb[5];
                    rn[6 * TILE_X + lane - 1] = fb[6];
                }
                if (walls && c == 0) {
                    r0[2 * TILE_X + lane] = fb[4];
                    r0[5 * TILE_X + lane] = fb[7];
                    r0[6 * TILE_X + lane] = fb[8];
                } else {
                    T *rs = f1row(c - 1);
                    rs[4 * TILE_X + lane] = fb[4];
                    rs[7 * TILE_X + lane - 1] = fb[7];
                    rs[8 * TILE_X + lane + 1] = fb[8];
                }
            }
        }

        // step t + 1: rho and psi of a completed LDS row (ghost rows beyond a
        // wall mirror the wall row)
        const int rb = rowB(k - 4);
        if (!single && k >= 4 && rb <= y_end) {
            const int rr = walls ? min(max(rb, 0), ny - 1) : rb;
            const T *src = f1row(rr);
#pragma unroll
            for (int a = 0; a < 9; ++a) gn[a] = src[a * TILE_X + lane];
            T ps = T(0);
            if (lane_b) {
                const T dm = density<T>(gn);
                ps = pseudopotential<T, EOS64>(dm, d);
                bad |= !finite_value(ps);
                if (track && (rb == 0 || rb == ny - 1) && rb >= tl.y0 && rb < y_end && out)
                    wmaxB = fmax(wmaxB, eos_pressure<double>(d.rho_ref + (double)dm, d.RT, d.a, d.b4));
            }
            psiB[(rb & (RP - 1)) * TILE_X + lane] = ps;
        }

        // step t + 1: collide the row read two iterations ago, to memory
        const int cb = rowB(k - 6);
        if (!single && k >= 6 && cb >= tl.y0 && cb < y_end && out) {
            const T *rS = psiB + ((cb - 1) & (RP - 1)) * TILE_X;
            const T *rC = psiB + (cb & (RP - 1)) * TILE_X;
            const T *rN = psiB + ((cb + 1) & (RP - 1)) * TILE_X;
            T pc, Fx, Fy;
            interaction_force<T>(rS, rC, rN, lane, mG, pc, Fx, Fy);
            collide_site<T>(gb, pc, Fx, Fy, R, cw ^ row_word(cb, ny, swB));
            if (write_through) push_store<T, true>(fo, PB, gb, xo, xeo, xwo, cb, ny, RB, walls);
            else push_store<T>(fo, PB, gb, xo, xeo, xwo, cb, ny, RB, walls);
        }

        __syncthreads();
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            fb[a] = fa[a];
            fa[a] = fn[a];
            if (next) fn[a] = fq[a];
            gb[a] = ga[a];
            ga[a] = gn[a];
        }
        mb = ma;
        ma = mn;
        if (next) mn = mq;
    };

#pragma unroll 2
    for (int k = 0; k < NA - 1; ++k) iteration(k, true);
    for (int k = NA - 1; k < NK; ++k) iteration(k, false);
    if (bad) d.flag[0] = 1;
    if (track) {
        // the population ring is free after the walk's last barrier
        double *red = reinterpret_cast<double *>(f1);
        red[threadIdx.x] = wmaxA;
        red[BLOCK + threadIdx.x] = wmaxB;
        __syncthreads();
        for (int k2 = BLOCK / 2; k2 > 0; k2 >>= 1) {
            if (threadIdx.x < k2) {
                red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k2]);
                red[BLOCK + threadIdx.x] = fmax(red[BLOCK + threadIdx.x], red[BLOCK + threadIdx.x + k2]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (red[0] > -INFINITY) atomicMax(&d.wall_keys[2 * s], order_key(red[0]));
            if (!single && red[BLOCK] > -INFINITY) atomicMax(&d.wall_keys[2 * s + 1], order_key(red[BLOCK]));
        }
    }
}

// ---------------------------------------------------------------------------
// end of a chunk: fold the per-step wall maxima, advance step counter/parity
// ---------------------------------------------------------------------------
__global__ void chunk_end_kernel(InstDev *insts, int ninst, int *status, int pairs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst) return;
    InstDev &d = insts[k];
    if (status) status[k] = d.flag[0];          // the batch's copy of every latch
    const int n = d.n_chunk;
    if (n <= 0) return;
    if (d.walls) {
        unsigned long long best = d.wall_run[0];
        long long best_step = (long long)d.wall_run[1];
        for (int j = 0; j < n; ++j) {
            const unsigned long long key = d.wall_keys[j];
            if (key > best) {
                best = key;
                best_step = d.step + j;
            }
            d.wall_keys[j] = 0ull;
        }
        d.wall_run[0] = best;
        d.wall_run[1] = (unsigned long long)best_step;
    }
    d.step += n;
    d.cur ^= buffer_flips(n, pairs) & 1;
}

// Clears the latch and the wall-pressure record of one instance.
__global__ void reset_diag_kernel(const InstDev *inst)
{
    const InstDev &d = *inst;
    for (int j = threadIdx.x; j < MAX_CHUNK; j += blockDim.x) d.wall_keys[j] = 0ull;
    if (threadIdx.x == 0) {
        d.wall_run[0] = 0ull;
        d.wall_run[1] = 0ull;
        d.flag[0] = 0;
    }
}

// ---------------------------------------------------------------------------
// initial state (Eq. 16), f_a = w_a rho
// ---------------------------------------------------------------------------
struct InitArgs {
    int slab_rows, nb;
    double rho_l, rho_g, W, delta, noise_amp;
    unsigned long long seed;
    double bx[LBM_MAX_BUBBLES], by[LBM_MAX_BUBBLES], br[LBM_MAX_BUBBLES];
};

// SplitMix64 (Steele, Lea and Flood): one output for the state s.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long s)
{
    unsigned long long z = s + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void init_kernel(const InstDev *inst, InitArgs A)
{
    const InstDev &d = *inst;
    const long long n = (long long)d.nx * d.ny;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = (int)(i / d.nx);
    const int x = (int)(i - (long long)y * d.nx);
    const double rl = A.rho_l * (1.0 + A.delta);
    double dist;                                // positive on the liquid side
    if (A.slab_rows > 0) {
        dist = 0.5 * A.slab_rows - fabs(y - 0.5 * (d.ny - 1));
    } else {
        dist = INFINITY;
        for (int k = 0; k < A.nb; ++k) {
            const double dx = x - A.bx[k], dy = y - A.by[k];
            dist = fmin(dist, sqrt(dx * dx + dy * dy) - A.br[k]);
        }
    }
    double rho = 0.5 * (rl + A.rho_g) + 0.5 * (rl - A.rho_g) * tanh(2.0 * dist / A.W);
    if (A.noise_amp != 0.0) {
        const double u = (double)(splitmix64(A.seed ^ (unsigned long long)i) >> 11) *
                         (1.0 / 9007199254740992.0);
        rho *= 1.0 + A.noise_amp * (2.0 * u - 1.0);
    }
    T *f = (T *)d.f[d.cur];
    const long long j = (long long)y * d.pitch + x;
    const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w5 = 1.0 / 36.0;
    const double dev = rho - d.rho_ref;        // stored shifted by w_a rho_ref
    f[j] = (T)(w0 * dev);
#pragma unroll
    for (int a = 1; a <= 4; ++a) f[a * d.plane + j] = (T)(w1 * dev);
#pragma unroll
    for (int a = 5; a <= 8; ++a) f[a * d.plane + j] = (T)(w5 * dev);
}

// f_a = w_a rho from a dense binary64 density field
template <typename T>
__global__ void init_density_kernel(const InstDev *inst, const double *__restrict__ rho_in)
{
    const InstDev &d = *inst;
    const long long n = (long long)d.nx * d.ny;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = (int)(i / d.nx);
    const int x = (int)(i - (long long)y * d.nx);
    const double dev = rho_in[i] - d.rho_ref;
    T *f = (T *)d.f[d.cur];
    const long long j = (long long)y * d.pitch + x;
    f[j] = (T)(4.0 / 9.0 * dev);
#pragma unroll
    for (int a = 1; a <= 4; ++a) f[a * d.plane + j] = (T)(1.0 / 9.0 * dev);
#pragma unroll
    for (int a = 5; a <= 8; ++a) f[a * d.plane + j] = (T)(1.0 / 36.0 * dev);
}

// ---------------------------------------------------------------------------
// macroscopic fields and per-tile binary64 partial sums
// ---------------------------------------------------------------------------
template <typename T, int RY>
__global__ __launch_bounds__(BLOCK) void macros_kernel(const InstDev *__restrict__ insts,
                                                       const Tile *__restrict__ tiles, int ntiles,
                                                       T *rho_out, T *ux_out, T *uy_out,
                                                       double *p_out)
{
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const InstDev &d = insts[tl.inst];
    const T *__restrict__ f = (const T *)d.f[d.cur];
    const T *__restrict__ psi = (const T *)d.psi;
    const long long P = d.plane;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int lx = threadIdx.x & (TILE_X - 1);
    const int g = threadIdx.x / TILE_X;
    const int x = tl.x0 + lx;

    double acc[N_PARTIAL];
#pragma unroll
    for (int q = 0; q < N_PARTIAL; ++q) acc[q] = 0.0;

    for (int r = 0; r < RY; ++r) {
        const int y = tl.y0 + g * RY + r;
        if (x >= nx || y >= ny) continue;
        const long long i = (long long)y * pitch + x;
        T v[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) v[a] = f[a * P + i];
        const T dm = density<T>(v);
        const T rho = consts<T>(d).rho_ref + dm;
        const T jx = momentum_x<T>(v);
        const T jy = momentum_y<T>(v);
        auto ps = [&](int dx, int dy) -> T {
            int xx = x + dx;
            xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
            int yy = y + dy;
            if (d.walls) yy = yy < 0 ? 0 : (yy > ny - 1 ? ny - 1 : yy);
            else yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
            return psi[(long long)yy * pitch + xx];
        };
        const T pc = ps(0, 0);
        // as in interaction_force()
        const T gx = fma(T(1.0 / 12.0), (ps(1, 1) - ps(-1, 1)) + (ps(1, -1) - ps(-1, -1)),
                         T(1.0 / 3.0) * (ps(1, 0) - ps(-1, 0)));
        const T gy = fma(T(1.0 / 12.0), (ps(1, 1) + ps(-1, 1)) - (ps(1, -1) + ps(-1, -1)),
                         T(1.0 / 3.0) * (ps(0, 1) - ps(0, -1)));
        const T mG = consts<T>(d).mG;
        const T Fx = mG * pc * gx, Fy = mG * pc * gy;
        const T mx = jx + T(0.5) * Fx, my = jy + T(0.5) * Fy;
        const long long o = (long long)y * nx + x;
        if (rho_out) rho_out[o] = rho;
        if (ux_out) ux_out[o] = mx / rho;
        if (uy_out) uy_out[o] = my / rho;
        if (p_out) p_out[o] = eos_pressure<double>(d.rho_ref + (double)dm, d.RT, d.a, d.b4);
        acc[0] += d.rho_ref + (double)dm;
        acc[1] += (double)mx;
        acc[2] += (double)my;
        if (d.n_bubbles > 0) {
            double frac = (d.rho_l - (d.rho_ref + (double)dm)) / (d.rho_l - d.rho_g);
            frac = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
            int best = 0;
            double bd = INFINITY;
            for (int k = 0; k < d.n_bubbles; ++k) {
                const double dx = x - d.bx[k], dy = y - d.by[k];
                const double dd = dx * dx + dy * dy;
                if (dd < bd) { bd = dd; best = k; }
            }
#pragma unroll
            for (int k = 0; k < LBM_MAX_BUBBLES; ++k)
                if (k == best) acc[3 + k] += frac;
        }
    }
    __shared__ double red[BLOCK];
    for (int q = 0; q < N_PARTIAL; ++q) {
        red[threadIdx.x] = acc[q];
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) d.partials[(long long)q * ntiles + tl.tile_index] = red[0];
        __syncthreads();
    }
}

// Sums the per-tile partials of one instance in a fixed order.
__global__ void reduce_kernel(const InstDev *inst, int ntiles)
{
    const InstDev &d = *inst;
    __shared__ double red[BLOCK];
    for (int q = 0; q < N_PARTIAL; ++q) {
        double acc = 0.0;
        for (int k = threadIdx.x; k < ntiles; k += BLOCK) acc += d.partials[(long long)q * ntiles + k];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) d.result[q] = red[0];
        __syncthreads();
    }
}

// Copies between the padded state buffer and a dense f[a][y][x] array.
template <typename T>
__global__ void pack_kernel(const InstDev *inst, T *dense, int to_dense)
{
    const InstDev &d = *inst;
    const long long n = (long long)d.nx * d.ny;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (i >= n) return;
    const int y = (int)(i / d.nx);
    const int x = (int)(i - (long long)y * d.nx);
    T *f = (T *)d.f[d.cur];
    const long long j = a * d.plane + (long long)y * d.pitch + x;
    // dense arrays hold plain populations; the state holds them shifted
    const double w = a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    if (to_dense) dense[a * n + i] = (T)((double)f[j] + w * d.rho_ref);
    else f[j] = (T)((double)dense[a * n + i] - w * d.rho_ref);
}

__global__ void copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

inline unsigned grid_for(int ntiles)
{
    return (unsigned)(((ntiles + NXCD - 1) / NXCD) * NXCD);
}

template <typename T, bool E64>
hipError_t psi_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, int s, hipStream_t st)
{
    const dim3 grid(grid_for(nt)), block(BLOCK);
    switch (kVariants[variant].rows) {
    case 1: psi_pass_kernel<T, E64, 1><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 2: psi_pass_kernel<T, E64, 2><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 4: psi_pass_kernel<T, E64, 4><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 8: psi_pass_kernel<T, E64, 8><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t collide_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, int s,
                            hipStream_t st)
{
    const dim3 grid(grid_for(nt)), block(BLOCK);
    switch (kVariants[variant].rows) {
    case 1: collide_stream_kernel<T, 1><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 2: collide_stream_kernel<T, 2><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 4: collide_stream_kernel<T, 4><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    case 8: collide_stream_kernel<T, 8><<<grid, block, 0, st>>>(di, dt, nt, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool E64>
hipError_t fused_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, int s, int alt,
                          int wt, hipStream_t st)
{
    const dim3 grid(grid_for(nt)), block(BLOCK);
    switch (kVariants[variant].rows) {
    case 16: fused_kernel<T, E64, 16><<<grid, block, 0, st>>>(di, dt, nt, s, alt, wt); break;
    case 32: fused_kernel<T, E64, 32><<<grid, block, 0, st>>>(di, dt, nt, s, alt, wt); break;
    case 64: fused_kernel<T, E64, 64><<<grid, block, 0, st>>>(di, dt, nt, s, alt, wt); break;
    case 128: fused_kernel<T, E64, 128><<<grid, block, 0, st>>>(di, dt, nt, s, alt, wt); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool E64>
hipError_t fused2_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, int s, int alt,
                           hipStream_t st)
{
    const dim3 grid(grid_for(nt)), block(BLOCK);
    switch (kVariants[variant].rows) {
    case 16: fused2_kernel<T, E64, 16><<<grid, block, 0, st>>>(di, dt, nt, s, alt); break;
    case 32: fused2_kernel<T, E64, 32><<<grid, block, 0, st>>>(di, dt, nt, s, alt); break;
    case 64: fused2_kernel<T, E64, 64><<<grid, block, 0, st>>>(di, dt, nt, s, alt); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool E64>
hipError_t twostep_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, int s, int wt,
                            hipStream_t st)
{
    const dim3 grid(grid_for(nt)), block(BLOCK);
    switch (kVariants[variant].rows) {
    case 16: twostep_kernel<T, E64, 16><<<grid, block, 0, st>>>(di, dt, nt, s, wt); break;
    case 24: twostep_kernel<T, E64, 24><<<grid, block, 0, st>>>(di, dt, nt, s, wt); break;
    case 32: twostep_kernel<T, E64, 32><<<grid, block, 0, st>>>(di, dt, nt, s, wt); break;
    case 48: twostep_kernel<T, E64, 48><<<grid, block, 0, st>>>(di, dt, nt, s, wt); break;
    case 64: twostep_kernel<T, E64, 64><<<grid, block, 0, st>>>(di, dt, nt, s, wt); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Fused instantiation of a variant (nullptr for the two-pass variants).
template <typename T, bool E64>
const void *fused_ptr(int variant)
{
    const Variant &v = kVariants[variant];
    if (v.fused == 1) {
        switch (v.rows) {
        case 16: return reinterpret_cast<const void *>(fused_kernel<T, E64, 16>);
        case 32: return reinterpret_cast<const void *>(fused_kernel<T, E64, 32>);
        case 64: return reinterpret_cast<const void *>(fused_kernel<T, E64, 64>);
        case 128: return reinterpret_cast<const void *>(fused_kernel<T, E64, 128>);
        default: return nullptr;
        }
    }
    if (v.fused == 2) {
        switch (v.rows) {
        case 16: return reinterpret_cast<const void *>(fused2_kernel<T, E64, 16>);
        case 32: return reinterpret_cast<const void *>(fused2_kernel<T, E64, 32>);
        case 64: return reinterpret_cast<const void *>(fused2_kernel<T, E64, 64>);
        default: return nullptr;
        }
    }
    return nullptr;
}

// Blocks of each fused instantiation that the device holds at once, by
// precision mode and variant (0: not known), filled once by
// prime_residency() outside any graph capture (the occupancy query is a
// runtime call).  Only the walk order of the fused kernels depends on it.
// Atomic so that lbm_resident_blocks may read it from any thread.
constexpr int kMaxVariants = 16;
std::atomic<int> g_resident[3][kMaxVariants];
std::once_flag g_resident_once;

int whole_grid_resident(int prec, int variant, int ntiles)
{
    if (prec < 0 || prec > 2 || variant < 0 || variant >= kMaxVariants) return 0;
    return (long long)grid_for(ntiles) <= (long long)g_resident[prec][variant].load(std::memory_order_relaxed)
               ? 1 : 0;
}

template <typename T>
hipError_t macros_dispatch(int variant, const InstDev *di, const Tile *dt, int nt, void *rho,
                           void *ux, void *uy, double *p, hipStream_t st)
{
    const dim3 grid(nt), block(BLOCK);
    T *r = (T *)rho, *u = (T *)ux, *v = (T *)uy;
    switch (kVariants[variant].rows) {
    case 1: macros_kernel<T, 1><<<grid, block, 0, st>>>(di, dt, nt, r, u, v, p); break;
    case 2: macros_kernel<T, 2><<<grid, block, 0, st>>>(di, dt, nt, r, u, v, p); break;
    case 4: macros_kernel<T, 4><<<grid, block, 0, st>>>(di, dt, nt, r, u, v, p); break;
    case 8: macros_kernel<T, 8><<<grid, block, 0, st>>>(di, dt, nt, r, u, v, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_psi_pass(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                           int ntiles, int s, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (prec == LBM_FP64) return psi_dispatch<double, false>(variant, d_inst, d_tiles, ntiles, s, st);
    if (prec == LBM_FP32) return psi_dispatch<float, false>(variant, d_inst, d_tiles, ntiles, s, st);
    return psi_dispatch<float, true>(variant, d_inst, d_tiles, ntiles, s, st);
}

hipError_t launch_collide_stream(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                                 int ntiles, int s, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (prec == LBM_FP64) return collide_dispatch<double>(variant, d_inst, d_tiles, ntiles, s, st);
    return collide_dispatch<float>(variant, d_inst, d_tiles, ntiles, s, st);
}

int resident_blocks(int prec, int variant)
{
    if (prec < 0 || prec > 2 || variant < 0 || variant >= kMaxVariants) return 0;
    return g_resident[prec][variant].load(std::memory_order_relaxed);
}

void prime_residency()
{
    std::call_once(g_resident_once, [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        for (int v = 0; v < kNumVariants && v < kMaxVariants; ++v)
            for (int p = 0; p < 3; ++p) {
                const void *k = p == LBM_FP64   ? fused_ptr<double, false>(v)
                                : p == LBM_FP32 ? fused_ptr<float, false>(v)
                                                : fused_ptr<float, true>(v);
                int per_cu = 0;
                if (!k) continue;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, BLOCK, 0) == hipSuccess)
                    g_resident[p][v].store(per_cu * cus, std::memory_order_relaxed);
                else
                    (void)hipGetLastError();
            }
    });
}

hipError_t launch_fused(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                        int s, hipStream_t st, int write_through)
{
    if (ntiles <= 0) return hipSuccess;
    if (kVariants[variant].fused != 1) return hipErrorInvalidValue;
    const int alt = whole_grid_resident(prec, variant, ntiles);
    const int wt = write_through ? 1 : 0;
    if (prec == LBM_FP64) return fused_dispatch<double, false>(variant, d_inst, d_tiles, ntiles, s, alt, wt, st);
    if (prec == LBM_FP32) return fused_dispatch<float, false>(variant, d_inst, d_tiles, ntiles, s, alt, wt, st);
    return fused_dispatch<float, true>(variant, d_inst, d_tiles, ntiles, s, alt, wt, st);
}

hipError_t launch_fused2(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                         int s, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (kVariants[variant].fused != 2) return hipErrorInvalidValue;
    const int alt = whole_grid_resident(prec, variant, ntiles);
    if (prec == LBM_FP64) return fused2_dispatch<double, false>(variant, d_inst, d_tiles, ntiles, s, alt, st);
    if (prec == LBM_FP32) return fused2_dispatch<float, false>(variant, d_inst, d_tiles, ntiles, s, alt, st);
    return fused2_dispatch<float, true>(variant, d_inst, d_tiles, ntiles, s, alt, st);
}

hipError_t launch_twostep(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles, int ntiles,
                          int s, hipStream_t st, int write_through)
{
    if (ntiles <= 0) return hipSuccess;
    if (kVariants[variant].fused != 3) return hipErrorInvalidValue;
    const int wt = write_through ? 1 : 0;
    if (prec == LBM_FP64) return twostep_dispatch<double, false>(variant, d_inst, d_tiles, ntiles, s, wt, st);
    if (prec == LBM_FP32) return twostep_dispatch<float, false>(variant, d_inst, d_tiles, ntiles, s, wt, st);
    return twostep_dispatch<float, true>(variant, d_inst, d_tiles, ntiles, s, wt, st);
}

hipError_t launch_chunk_end(const InstDev *d_inst, int ninst, hipStream_t st, int *d_status, int pairs)
{
    if (ninst <= 0) return hipSuccess;
    chunk_end_kernel<<<(ninst + 63) / 64, 64, 0, st>>>(const_cast<InstDev *>(d_inst), ninst, d_status, pairs);
    return hipGetLastError();
}

hipError_t launch_reset_diag(const InstDev *d_inst, hipStream_t st)
{
    reset_diag_kernel<<<1, 256, 0, st>>>(d_inst);
    return hipGetLastError();
}

hipError_t launch_init(int prec, const InstDev *d_inst, int slab_rows, const lbm_bubble *b, int nb,
                       double rho_l, double rho_g, double W, double delta, double noise_amp,
                       uint64_t seed, long long nsites, hipStream_t st)
{
    InitArgs A;
    A.slab_rows = slab_rows;
    A.nb = nb;
    A.rho_l = rho_l;
    A.rho_g = rho_g;
    A.W = W;
    A.delta = delta;
    A.noise_amp = noise_amp;
    A.seed = seed;
    for (int k = 0; k < LBM_MAX_BUBBLES; ++k) {
        A.bx[k] = k < nb ? b[k].x0 : 0.0;
        A.by[k] = k < nb ? b[k].y0 : 0.0;
        A.br[k] = k < nb ? b[k].r0 : 0.0;
    }
    const unsigned grid = (unsigned)((nsites + 255) / 256);
    if (prec == LBM_FP64) init_kernel<double><<<grid, 256, 0, st>>>(d_inst, A);
    else init_kernel<float><<<grid, 256, 0, st>>>(d_inst, A);
    return hipGetLastError();
}

hipError_t launch_init_density(int prec, const InstDev *d_inst, const double *rho, long long nsites,
                              hipStream_t st)
{
    const unsigned grid = (unsigned)((nsites + 255) / 256);
    if (prec == LBM_FP64) init_density_kernel<double><<<grid, 256, 0, st>>>(d_inst, rho);
    else init_density_kernel<float><<<grid, 256, 0, st>>>(d_inst, rho);
    return hipGetLastError();
}

hipError_t launch_macros(int prec, int variant, const InstDev *d_inst, const Tile *d_tiles,
                         int ntiles, void *rho, void *ux, void *uy, double *p, hipStream_t st)
{
    if (prec == LBM_FP64) return macros_dispatch<double>(variant, d_inst, d_tiles, ntiles, rho, ux, uy, p, st);
    return macros_dispatch<float>(variant, d_inst, d_tiles, ntiles, rho, ux, uy, p, st);
}

hipError_t launch_reduce(const InstDev *d_inst, int ntiles, hipStream_t st)
{
    reduce_kernel<<<1, BLOCK, 0, st>>>(d_inst, ntiles);
    return hipGetLastError();
}

hipError_t launch_pack(int prec, const InstDev *d_inst, int nx, int ny, void *dense, int to_dense,
                       hipStream_t st)
{
    const long long n = (long long)nx * ny;
    const dim3 grid((unsigned)((n + 255) / 256), 9);
    if (prec == LBM_FP64) pack_kernel<double><<<grid, 256, 0, st>>>(d_inst, (double *)dense, to_dense);
    else pack_kernel<float><<<grid, 256, 0, st>>>(d_inst, (float *)dense, to_dense);
    return hipGetLastError();
}

__global__ void fill_int_kernel(int *dst, int n, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

hipError_t launch_fill_int(int *dst, int n, int value, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    fill_int_kernel<<<(n + 255) / 256, 256, 0, st>>>(dst, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t n, hipStream_t st)
{
    const size_t n16 = n / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    copy_kernel<<<(unsigned)blocks, 256, 0, st>>>((uint4 *)dst, (const uint4 *)src, n16);
    return hipGetLastError();
}

}  // namespace lbm
