// Checks of the library's GPU-free host logic (paper_2006_10004_amd/csrc/
// host_logic.cpp), built by tests/test_host_sanitized.py with g++ and the
// address and undefined-behaviour sanitizers:
//   - argument validation on edge and adversarial values (limits, overflow
//     bait, non-finite numbers) returns the documented codes;
//   - band_rows_of against the band definition on random edge sets;
//   - RangeAlloc against a shadow model over random alloc / release
//     sequences: no two live ranges overlap, every range lies in the pool,
//     used() is the sum of the live aligned sizes, peak() its maximum, and
//     releasing everything leaves one free range of the whole pool.
// Prints "host logic ok" and returns 0, or names the failed check.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "host_logic.h"

using namespace tvspec;

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);  \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static void check_validation()
{
    const int I = INT_MAX;
    CHECK(validate_shape(1, 2, 2, 1, 1) == TVSPEC_OK);
    CHECK(validate_shape(0, 8, 8, 1, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(-1, 8, 8, 1, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 1, 8, 1, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 8, 1, 1, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 8, 8, 0, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 8, 8, 1, 0) == TVSPEC_EINVAL);
    CHECK(validate_shape(I, 8, 8, I, 1) == TVSPEC_EINVAL);   // B*C overflow bait
    CHECK(validate_shape(1, I, I, 1, 1) == TVSPEC_EINVAL);   // H*W overflow bait
    CHECK(validate_shape(255, 1 << 15, 1 << 15, 257, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 1 << 15, 1 << 15, 1, 1) == TVSPEC_OK);
    CHECK(validate_shape(65535, 2, 2, 1, 1) == TVSPEC_OK);
    CHECK(validate_shape(65536, 2, 2, 1, 1) == TVSPEC_EINVAL);
    CHECK(validate_shape(1, 1 << 15, 1 << 15, 1024, 1) == TVSPEC_OK);      // 2^40 pixels
    CHECK(validate_shape(1, 1 << 15, 1 << 15, 1025, 1) == TVSPEC_EINVAL);  // > 2^40 pixels
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    const int e4[] = {0, 1, 2, 4};
    CHECK(validate_image(0.01, 4, e4, 3) == TVSPEC_OK);
    CHECK(validate_image(nan, 4, e4, 3) == TVSPEC_EINVAL);
    CHECK(validate_image(inf, 4, e4, 3) == TVSPEC_EINVAL);
    CHECK(validate_image(-0.0, 4, e4, 3) == TVSPEC_EINVAL);
    CHECK(validate_image(0.01, 0, e4, 3) == TVSPEC_EINVAL);
    CHECK(validate_image(0.01, 5, e4, 3) == TVSPEC_EINVAL);  // last edge != K
    CHECK(validate_image(0.01, 4, e4, 0) == TVSPEC_EINVAL);
    CHECK(validate_image(0.01, 2, e4, 3) == TVSPEC_EINVAL);  // more bands than samples
    const int dup[] = {0, 2, 2, 4};
    CHECK(validate_image(0.01, 4, dup, 3) == TVSPEC_EINVAL);
    const int neg[] = {-1, 2, 3, 4};
    CHECK(validate_image(0.01, 4, neg, 3) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.248, 0, TVSPEC_PRECISION_MIXED, 0) == TVSPEC_OK);
    CHECK(validate_opts(0.25, 1, TVSPEC_PRECISION_F32, 16) == TVSPEC_OK);
    CHECK(validate_opts(0.2500001, 0, TVSPEC_PRECISION_F32, 0) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.0, 0, TVSPEC_PRECISION_F32, 0) == TVSPEC_EINVAL);
    CHECK(validate_opts(nan, 0, TVSPEC_PRECISION_F32, 0) == TVSPEC_EINVAL);
    CHECK(validate_tile_shape(TVSPEC_TILE_SQUARE, TVSPEC_SOLVER_PDHG, 16) == TVSPEC_OK);
    CHECK(validate_tile_shape(TVSPEC_TILE_NARROW, TVSPEC_SOLVER_CHAMBOLLE, 8) == TVSPEC_OK);
    CHECK(validate_tile_shape(TVSPEC_TILE_NARROW, TVSPEC_SOLVER_CHAMBOLLE, 16) == TVSPEC_EINVAL);
    CHECK(validate_tile_shape(TVSPEC_TILE_NARROW, TVSPEC_SOLVER_PDHG, 0) == TVSPEC_EINVAL);
    CHECK(validate_tile_shape(2, TVSPEC_SOLVER_CHAMBOLLE, 0) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.1, 2, TVSPEC_PRECISION_F32, 0) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.1, 0, 3, 0) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.1, 0, TVSPEC_PRECISION_F64, 9) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.1, 0, TVSPEC_PRECISION_MIXED, -1) == TVSPEC_EINVAL);
    CHECK(validate_opts(0.1, 0, TVSPEC_PRECISION_F32, 17) == TVSPEC_EINVAL);
    g_last_error.clear();
    CHECK(fail(TVSPEC_EINVAL, "x") == TVSPEC_EINVAL && g_last_error == "x");
}

static void check_band_rows(std::mt19937_64 &rng)
{
    for (int trial = 0; trial < 2000; ++trial) {
        const int K = 1 + (int)(rng() % 400);
        const int nb = 1 + (int)(rng() % std::min(K, 12));
        // nb - 1 distinct interior edges in 1..K-1
        std::vector<int> e{0, K};
        while ((int)e.size() < nb + 1) {
            const int v = 1 + (int)(rng() % (unsigned)std::max(K - 1, 1));
            if (v < K && std::find(e.begin(), e.end(), v) == e.end())
                e.push_back(v);
        }
        std::sort(e.begin(), e.end());
        CHECK(validate_image(0.01, K, e.data(), nb) == TVSPEC_OK);
        std::vector<int> rows(K + 1, -7);
        band_rows_of(e.data(), nb, rows.data());
        CHECK(rows[0] == 0);
        for (int k = 1; k <= K; ++k) {
            int want = -1;
            for (int j = 0; j < nb; ++j)
                if (e[j] < k && k <= e[j + 1])
                    want = j;
            CHECK(rows[k] == want);
        }
    }
}

static void check_range_alloc(std::mt19937_64 &rng)
{
    struct Live { size_t off, n; };
    for (int trial = 0; trial < 40; ++trial) {
        const size_t cap = align256((size_t)(1 + rng() % (64u << 20)));
        RangeAlloc a;
        a.reset(cap);
        std::vector<Live> live;
        size_t used = 0, peak = 0;
        for (int step = 0; step < 4000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t n = 1 + (size_t)(rng() % (cap / 8 + 1));
                size_t off = ~(size_t)0;
                if (a.alloc(n, &off)) {
                    const size_t an = align256(n);
                    CHECK(off % 256 == 0 && off + an <= cap);
                    for (const Live &l : live)
                        CHECK(off + an <= l.off || l.off + l.n <= off);
                    live.push_back({off, an});
                    used += an;
                    peak = std::max(peak, used);
                } else {
                    CHECK(!live.empty() || align256(n) > cap); // an empty pool fits anything up to cap
                }
            } else {
                const size_t i = (size_t)(rng() % live.size());
                a.release(live[i].off, live[i].n);
                used -= live[i].n;
                live[i] = live.back();
                live.pop_back();
            }
            CHECK(a.used() == used);
            CHECK(a.peak() == peak);
        }
        for (const Live &l : live)
            a.release(l.off, l.n);
        CHECK(a.used() == 0);
        size_t off = 1;
        CHECK(a.alloc(cap, &off) && off == 0); // one free range of the whole pool again
    }
}

int main()
{
    std::mt19937_64 rng(20060);
    check_validation();
    check_band_rows(rng);
    check_range_alloc(rng);
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("host logic ok\n");
    return 0;
}
