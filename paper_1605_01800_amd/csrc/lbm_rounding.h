// Stochastic rounding of the binary32 rest population (lbm_kernels.hip,
// collide_site) and the random words it draws.  Plain integer and binary32
// arithmetic, compiled for the device by hipcc and for the host by the unit
// test of the rounding (tests/test_rounding_host.py).
#pragma once

#if defined(__HIPCC__)
#define LBM_ROUNDING_FN __host__ __device__ __forceinline__
#else
#define LBM_ROUNDING_FN inline __attribute__((always_inline))
#endif

namespace lbm {

// lowbias32, the 32-bit integer hash of C. Wellons ("Prospecting for hash
// functions", 2018): xorshift-multiply rounds with his published constants.
LBM_ROUNDING_FN unsigned hash32(unsigned x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Random words of the stochastic rounding: site (x, y) (0 <= x < nx,
// 0 <= y < ny) in the step with word hash32(step) draws
// column_word(x) ^ row_word(y, step word).  Sites that the reflections of
// the grid through its centre (x -> nx - 1 - x, y -> ny - 1 - y) map onto
// each other draw the same word, so a mirror-symmetric state stays symmetric
// bit for bit, as with the mirror-symmetric sums.  The word depends on the
// instance's own step count and the site alone, not on tiles, batches or
// kernels, so every kernel family rounds every site alike.  A lane's column
// word is fixed for a launch and a row's is uniform over a wavefront (one
// scalar hash per row), so a site pays one exclusive or.
LBM_ROUNDING_FN unsigned column_word(int x, int nx)
{
    const int m = nx - 1 - x;
    return hash32((unsigned)(x < m ? x : m));
}

LBM_ROUNDING_FN unsigned row_word(int y, int ny, unsigned step_word)
{
    const int m = ny - 1 - y;
    return hash32((unsigned)(y < m ? y : m) ^ step_word);
}

// a + b rounded to one of the two binary32 values around it, the farther one
// with probability (distance to the nearer) / (gap between them), drawn from
// the top 24 bits of `key`: E[result] = a + b up to 2^-24 of the gap.  An
// exact sum is returned unchanged.  (TwoSum gives the exact error of the
// rounded sum; the neighbour toward it is one step of the encoding.)
LBM_ROUNDING_FN float stochastic_sum(float a, float b, unsigned key)
{
#pragma clang fp contract(off)
    const float s = a + b;
    const float bp = s - a;
    const float err = (a - (s - bp)) + (b - bp);               // a + b = s + err exactly
    const unsigned step = (err > 0.0f) == (s > 0.0f) ? 1u : ~0u;   // toward err, in the encoding
    const float o = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, s) + step);   // wraps
    const float gap = __builtin_fabsf(o - s);
    const float u = (float)(key >> 8) * 0x1p-24f;
    return u * gap < __builtin_fabsf(err) ? o : s;
}

}  // namespace lbm
