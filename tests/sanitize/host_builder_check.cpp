// Host-side SELL-C-sigma construction (the library's build.cpp, its thread pool included) run on
// random CSR matrices under AddressSanitizer / UndefinedBehaviorSanitizer or ThreadSanitizer.
// Besides the sanitizers' own checks it verifies the layout's invariants on every case: the
// permutation is a bijection onto the rows, chunk starts are the prefix sums of C times the chunk
// lengths, every row's entries (in order) and only padding (-1) fill its slot, and the tiles
// cover the chunks. Exit status 0 when every case holds.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "internal.h"

using namespace sellcs;

static int fail(const char *what, int64_t a, int64_t b) {
    std::fprintf(stderr, "FAIL %s (%lld, %lld)\n", what, (long long)a, (long long)b);
    return 1;
}

int main(int argc, char **argv) {
    const int reps = argc > 1 ? std::atoi(argv[1]) : 60;
    std::mt19937_64 rng(1507);
    int cases = 0;
    for (int rep = 0; rep < reps; ++rep) {
        const int64_t n = std::uniform_int_distribution<int64_t>(0, 3000)(rng);
        const int64_t ncols = std::uniform_int_distribution<int64_t>(1, 3000)(rng);
        std::vector<int64_t> rowptr(size_t(n) + 1, 0);
        std::vector<int32_t> col;
        std::vector<double> val;
        for (int64_t i = 0; i < n; ++i) {
            int64_t len = std::uniform_int_distribution<int64_t>(0, 12)(rng);
            if (rng() % 50 == 0) len = std::uniform_int_distribution<int64_t>(0, 400)(rng);  // long rows
            for (int64_t k = 0; k < len; ++k) {
                col.push_back(int32_t(rng() % uint64_t(ncols)));  // duplicates allowed
                val.push_back(std::uniform_real_distribution<double>(-1, 1)(rng));
            }
            rowptr[size_t(i) + 1] = int64_t(col.size());
        }
        const int32_t Cs[] = {1, 7, 32, 64};
        for (int32_t C : Cs) {
            const int64_t sigmas[] = {1, int64_t(C), 8 * int64_t(C), n > 0 ? n : 1, 1000000};
            for (int64_t sigma : sigmas) {
                const int vdt = int(rng() % 3);
                HostSell h;
                const int rc = build_host_sell(h, n, ncols, rowptr.data(), col.data(), val.data(), C,
                                               std::max<int64_t>(1, std::min<int64_t>(sigma, std::max<int64_t>(n, 1))),
                                               vdt);
                if (rc != SELL_OK) return fail("build", rc, 0);
                ++cases;
                const int64_t nslots = h.nch * C;
                if (h.nch != (n + C - 1) / C) return fail("nch", h.nch, n);
                if (int64_t(h.cs.size()) != h.nch + 1 || h.cs[0] != 0) return fail("cs size", int64_t(h.cs.size()), h.nch);
                for (int64_t c = 0; c < h.nch; ++c)
                    if (h.cs[size_t(c) + 1] - h.cs[size_t(c)] != int64_t(C) * h.cl[size_t(c)]) return fail("cs", c, 0);
                if (h.stored != h.cs[size_t(h.nch)]) return fail("stored", h.stored, h.cs[size_t(h.nch)]);
                std::vector<char> seen(size_t(n), 0);
                for (int64_t slot = 0; slot < nslots; ++slot) {
                    const int64_t row = h.has_perm ? h.perm[size_t(slot)] : (slot < n ? slot : -1);
                    const int64_t c = slot / C, r = slot % C;
                    const int64_t len = row >= 0 ? rowptr[size_t(row) + 1] - rowptr[size_t(row)] : 0;
                    if (row >= 0) {
                        if (row >= n || seen[size_t(row)]) return fail("perm", slot, row);
                        seen[size_t(row)] = 1;
                    }
                    if (len > h.cl[size_t(c)]) return fail("chunk length", c, len);
                    for (int64_t k = 0; k < h.cl[size_t(c)]; ++k) {
                        const int32_t got = h.col[size_t(h.cs[size_t(c)] + k * C + r)];
                        const int32_t want = k < len ? col[size_t(rowptr[size_t(row)] + k)] : -1;
                        if (got != want) return fail("entry", slot, k);
                    }
                }
                for (int64_t i = 0; i < n; ++i)
                    if (!seen[size_t(i)]) return fail("row missing", i, 0);
                if (h.tiles.empty() || h.tiles.front() != 0 || h.tiles.back() != h.nch) return fail("tiles", h.nch, 0);
                for (size_t t = 1; t < h.tiles.size(); ++t)
                    if (h.tiles[t] < h.tiles[t - 1]) return fail("tiles order", int64_t(t), 0);
            }
        }
    }
    std::printf("host builder: %d cases ok\n", cases);
    return 0;
}
