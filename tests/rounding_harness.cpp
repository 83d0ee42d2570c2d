// Host harness of the stochastic rounding (paper_1605_01800_amd/csrc/
// lbm_rounding.h) for tests/test_rounding_host.py.
//
//   rounding_harness sum A B        (A, B as hexadecimal binary32 bit patterns)
//     rounds A + B with every one of the 2^24 keys the rounding tells apart
//     and prints each value returned with the number of keys that returned
//     it (two at most), then the count of any further values
//   rounding_harness hash X         prints hash32(X)
//   rounding_harness words NX NY    checks that column_word / row_word are the
//     same for sites the grid's reflections map onto each other; prints ok
//   rounding_harness steps NX NY X Y N   histogram (256 bins) of the top byte
//     of site (X, Y)'s random word over steps 0 .. N-1
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "lbm_rounding.h"

static float from_bits(unsigned u) { return __builtin_bit_cast(float, u); }
static unsigned to_bits(float f) { return __builtin_bit_cast(unsigned, f); }

int main(int argc, char **argv)
{
    if (argc == 4 && !strcmp(argv[1], "sum")) {
        const float a = from_bits((unsigned)strtoul(argv[2], nullptr, 16));
        const float b = from_bits((unsigned)strtoul(argv[3], nullptr, 16));
        // every key k << 8, k < 2^24 (the rounding reads the top 24 bits)
        unsigned v[2] = {0, 0}, n[2] = {0, 0}, others = 0;
        for (unsigned k = 0; k < (1u << 24); ++k) {
            const unsigned r = to_bits(lbm::stochastic_sum(a, b, k << 8));
            if (n[0] == 0 || r == v[0]) { v[0] = r; ++n[0]; }
            else if (n[1] == 0 || r == v[1]) { v[1] = r; ++n[1]; }
            else ++others;                                         // a third value: an error
        }
        printf("%08x %u %08x %u %u\n", v[0], n[0], v[1], n[1], others);
        return 0;
    }
    if (argc == 3 && !strcmp(argv[1], "hash")) {
        printf("%08x\n", lbm::hash32((unsigned)strtoul(argv[2], nullptr, 0)));
        return 0;
    }
    if (argc == 4 && !strcmp(argv[1], "words")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]);
        for (int x = 0; x < nx; ++x)
            if (lbm::column_word(x, nx) != lbm::column_word(nx - 1 - x, nx)) { printf("column %d\n", x); return 1; }
        for (unsigned sw : {0u, 0x9e3779b9u, lbm::hash32(12345u)})
            for (int y = 0; y < ny; ++y)
                if (lbm::row_word(y, ny, sw) != lbm::row_word(ny - 1 - y, ny, sw)) { printf("row %d\n", y); return 1; }
        printf("ok\n");
        return 0;
    }
    if (argc == 7 && !strcmp(argv[1], "steps")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]), x = atoi(argv[4]), y = atoi(argv[5]);
        const unsigned n = (unsigned)strtoul(argv[6], nullptr, 0);
        unsigned counts[256] = {0};
        for (unsigned step = 0; step < n; ++step)
            ++counts[(lbm::column_word(x, nx) ^ lbm::row_word(y, ny, lbm::hash32(step))) >> 24];
        for (int b = 0; b < 256; ++b) printf("%u%c", counts[b], b == 255 ? '\n' : ' ');
        return 0;
    }
    fprintf(stderr, "usage: rounding_harness sum A B | hash X | words NX NY | steps NX NY X Y N\n");
    return 2;
}
