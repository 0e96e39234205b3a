// Exhaustive host-side checks of the library's index maps (no device code):
//  * propagator table slots: every frequency class (lx, ly) in [0, M/4]^2 has
//    a slot below table_slots(M, N); with 4 | N the classes (lx, ly) and
//    (ly, lx) share one slot, read through the reflection exactly when
//    lx > ly, and table_slot_class inverts the map on the stored order
//    (lx <= ly); otherwise every class has a slot of its own;
//  * the row-blocked layout: row_blk_index(kx, ky, C) is a bijection of
//    [0, C) x [0, M) onto [0, C M).
// Prints "bad <count>" and exits with 1 when any check fails.
#include <cstdio>
#include <vector>

#include "se2n_internal.hpp"

using namespace se2n;

int main() {
    long bad = 0, checked = 0;
    const int sides[] = {8, 12, 16, 20, 36, 64, 108, 324, 512, 1024, 2048, 4096};
    const int counts[] = {4, 5, 6, 8, 30, 31, 32, 64};
    for (int M : sides) {
        const int Q = M / 4 + 1;
        for (int N : counts) {
            const bool sym = table_sym(N);
            const size_t S = table_slots(M, N);
            if (S != (sym ? (size_t)Q * (Q + 1) / 2 : (size_t)Q * Q)) ++bad;
            std::vector<int> seen(S, 0);
            for (int lx = 0; lx < Q; ++lx) {
                for (int ly = 0; ly < Q; ++ly) {
                    ++checked;
                    const size_t s = table_slot(lx, ly, Q, N);
                    if (s >= S) { ++bad; continue; }
                    if (table_transposed(lx, ly, N) != (sym && lx > ly)) ++bad;
                    if (sym && lx > ly) {
                        if (s != table_slot(ly, lx, Q, N)) ++bad;
                        continue;
                    }
                    ++seen[s];
                    int a = -1, b = -1;
                    table_slot_class(s, Q, N, a, b);
                    if (a != lx || b != ly) ++bad;
                }
            }
            for (size_t s = 0; s < S; ++s)
                if (seen[s] != 1) ++bad;
        }
        for (int C : {M / 2, M / 2 + 1}) {
            if (M % kRowBlk) continue;
            std::vector<char> hit((size_t)C * M, 0);
            for (int ky = 0; ky < M; ++ky)
                for (int kx = 0; kx < C; ++kx) {
                    const long i = row_blk_index(kx, ky, C);
                    if (i < 0 || i >= (long)C * M || hit[i]) { ++bad; continue; }
                    hit[i] = 1;
                }
        }
    }
    std::printf("checked %ld classes, bad %ld\n", checked, bad);
    return bad ? 1 : 0;
}
