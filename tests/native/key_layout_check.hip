// Host-side check of the library's cell-key arithmetic (the same header
// functions the kernels call): the exact 64-by-32-bit division against the
// compiler's native 64-bit division, and the pack / unpack round trip of
// bit-packed and mixed-radix layouts.  Exit status 0 = every check passed.
#include "../../paper_2605_20353_amd/csrc/gcp_internal.hpp"

#include <cstdio>
#include <random>

using namespace gcp;

static long g_checks = 0, g_bad = 0;

static void check_div(uint64_t x, uint32_t dv)
{
    uint32_t r = 0;
    const uint64_t q = divmod_u64_u32(x, dv, 1.0 / (double)dv, r);
    ++g_checks;
    if (q != x / dv || r != x % dv) {
        if (g_bad < 10) std::printf("divmod %llu / %u gave %llu rem %u\n", (unsigned long long)x, dv, (unsigned long long)q, r);
        ++g_bad;
    }
}

static KeyLayout layout(const int64_t* dims, int d, bool radix)
{
    KeyLayout L{};
    L.d = d;
    L.radix = radix ? 1 : 0;
    int total = 0;
    uint64_t stride = 1;
    for (int k = d - 1; k >= 0; --k) {
        int b = 0;
        while (b < 63 && (int64_t(1) << b) < dims[k]) ++b;
        L.shift[k] = total;
        L.mask[k] = (1ull << b) - 1;
        total += b;
        L.dims[k] = dims[k];
        L.stride[k] = stride;
        L.inv[k] = 1.0 / (double)dims[k];
        stride *= (uint64_t)dims[k];
    }
    return L;
}

int main()
{
    std::mt19937_64 rng(20353);
    const uint64_t xs[] = {0ull, 1ull, 2ull, 0xffffffffull, 0x100000000ull, 0x1ffffffffull, ~0ull, ~0ull - 1,
                           1ull << 63, (1ull << 63) - 1, 15435000000000000000ull};
    const uint32_t ds[] = {1u, 2u, 3u, 7u, 100u, 65535u, 65536u, 4821207u, 1774269u, 1805187u,
                           0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu};
    for (uint64_t x : xs)
        for (uint32_t dv : ds) {
            check_div(x, dv);
            check_div(x + 1, dv);
            check_div(x - 1, dv);
        }
    // dividends next to exact multiples, where the double estimate is most
    // likely to land on the wrong side of an integer
    for (uint32_t dv : ds)
        for (uint64_t q : {1ull, 12345ull, 0xffffffffull, 0x100000001ull, (~0ull) / dv})
            for (int m = -3; m <= 3; ++m) {
                const unsigned __int128 v = (unsigned __int128)q * dv + (__int128)m;
                if (v <= (unsigned __int128)~0ull) check_div((uint64_t)v, dv);
            }
    for (long i = 0; i < 3000000; ++i) {
        const uint64_t x = rng() >> (rng() % 64);
        uint32_t dv = (uint32_t)(rng() >> (32 + rng() % 32));
        check_div(x, dv ? dv : 1u);
    }
    std::printf("divmod: %ld checks, %ld wrong\n", g_checks, g_bad);

    const int64_t shapes[][4] = {{4821207, 1774269, 1805187, 0}, {40000, 40000, 40000, 40000},
                                 {3, 5, 7, 11}, {10000, 8000, 6000, 0}};
    const int orders[] = {3, 4, 4, 3};
    long bad_keys = 0;
    for (int t = 0; t < 4; ++t) {
        for (int radix = 0; radix < 2; ++radix) {
            const KeyLayout L = layout(shapes[t], orders[t], radix != 0);
            int bits = 0;
            for (int k = 0; k < orders[t]; ++k) bits += __builtin_popcountll(L.mask[k]);
            if (!radix && bits > 63) continue;
            for (long i = 0; i < 300000; ++i) {
                uint32_t c[kMaxModes] = {}, u[kMaxModes] = {};
                uint64_t key = 0;
                for (int k = 0; k < orders[t]; ++k) {
                    uint64_t v = rng() % (uint64_t)L.dims[k];
                    if (i < 16) v = ((i >> (k % 4)) & 1) ? (uint64_t)L.dims[k] - 1 : 0;   // corners
                    c[k] = (uint32_t)v;
                    key += pack_coord(L, v, k);
                }
                if (key == kEmptySlot) ++bad_keys;
                unpack_all<true>(L, orders[t], key, u);
                for (int k = 0; k < orders[t]; ++k)
                    if (u[k] != c[k]) {
                        ++bad_keys;
                        break;
                    }
            }
            std::printf("shape %d, %s: %d bits, wrong so far %ld\n", t, radix ? "mixed radix" : "bit-packed", bits,
                        bad_keys);
        }
    }
    return (g_bad || bad_keys) ? 1 : 0;
}
