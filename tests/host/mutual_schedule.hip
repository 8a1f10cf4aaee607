// Host-side check of the each-pair-once passes' workgroup decode (built from
// the kernel source itself, run on the CPU): for every size, every range pair
// runs once, whole or as both halves (sub-phases 0-1 and 2-3, each over all
// its targets and sources), and every body receives each of its partial
// slots exactly once, with every slot inside the workspace.  The force pass
// and the transpose-Jacobian pass share this decode and these slot rules; the
// force pass's kernel-argument list of it decodes to the same.
#include "kernels_mutual.hip"
#include <cstdio>
#include <vector>
using namespace nb;
static int check(int64_t n, int tpl, int waves, bool verbose)
{
    const MutualTail tl = mutual_tail(n, tpl, waves);
    const int R = tl.R, S = mutual_slots(n, tpl, waves), nb = (int)((n + 63) / 64);
    if (S != R + 2 * tl.D) { printf("n=%ld slots %d R=%d D=%d\n", (long)n, S, R, tl.D); return 1; }
    const int64_t U = (int64_t)R * (R + 1) / 2;
    const int64_t grid = tl.F + 2 * (U - tl.F);
    std::vector<int> whole((size_t)R * R, 0), halves((size_t)R * R * 2, 0);
    std::vector<unsigned char> wr((size_t)n * S, 0);
    auto mark = [&](int64_t i, int slot) { if (i < n) { if (slot < 0 || slot >= S) { printf("slot %d of %d\n", slot, S); exit(1);} wr[(size_t)i * S + slot]++; } };
    // the kernel-argument list, where it applies, decodes to the same
    const MutualMap& map = mutual_map(tl, grid);
    if (map.count != 0 && (map.count != grid || R > 64 || grid > kMapMax)) { printf("n=%ld map count %d\n", (long)n, map.count); return 1; }
    if (map.count == 0 && R <= 64 && grid <= kMapMax) { printf("n=%ld map missing\n", (long)n); return 1; }
    for (int64_t b = 0; b < grid; ++b) {
        int g, r, half, xs;
        mt_decode(tl, b, g, r, half, xs);
        if (map.count > 0) {
            const unsigned v = map.e[b];
            const int mg = (int)(v & 63u), mr = (int)((v >> 6) & 63u), mh = (int)(v >> 12) - 1;
            const int mx = mh >= 0 ? R + (mr - mg) - 1 : 0;
            if (mg != g || mr != r || mh != half || (half >= 0 && mx != xs)) { printf("n=%ld b=%ld map differs\n", (long)n, (long)b); return 1; }
        }
        if (g < 0 || r < g || r >= R) { printf("n=%ld b=%ld bad (%d,%d)\n", (long)n, (long)b, g, r); return 1; }
        if (half < 0) {
            whole[(size_t)g * R + r]++;
            if (r > g) {
                for (int t = 0; t < 4; ++t) for (int l = 0; l < 64; ++l) mark((int64_t)(4 * g + t) * 64 + l, r);
                for (int jb = 0; jb < 4; ++jb) for (int l = 0; l < 64; ++l) mark((int64_t)(4 * r + jb) * 64 + l, g);
            } else {
                for (int t = 0; t < 4; ++t) for (int l = 0; l < 64; ++l) {
                    const int64_t i = (int64_t)(4 * g + t) * 64 + l;
                    mark(i, g);
                    for (int d = 1; d <= tl.D; ++d) {   // the diagonal workgroup's zeros
                        if (!mt_is_split(tl, g - d, d)) mark(i, tl.R + d - 1);
                        if (!mt_is_split(tl, g, d)) mark(i, tl.R + tl.D + d - 1);
                    }
                }
            }
        } else {
            if (r <= g) { printf("n=%ld split diagonal pair\n", (long)n); return 1; }
            halves[((size_t)g * R + r) * 2 + half]++;
            for (int t = 0; t < 4; ++t) for (int l = 0; l < 64; ++l) mark((int64_t)(4 * g + t) * 64 + l, half == 0 ? r : xs + tl.D);
            for (int jb = 0; jb < 4; ++jb) for (int l = 0; l < 64; ++l) mark((int64_t)(4 * r + jb) * 64 + l, half == 0 ? g : xs);
            if (half == 1 && (xs < R || xs >= S)) { printf("n=%ld xslot %d\n", (long)n, xs); return 1; }
        }
    }
    for (int g = 0; g < R; ++g) for (int r = g; r < R; ++r) {
        const int w = whole[(size_t)g * R + r], h0 = halves[((size_t)g * R + r) * 2], h1 = halves[((size_t)g * R + r) * 2 + 1];
        if (!((w == 1 && h0 == 0 && h1 == 0) || (w == 0 && h0 == 1 && h1 == 1))) { printf("n=%ld pair (%d,%d) whole %d halves %d %d\n", (long)n, g, r, w, h0, h1); return 1; }
    }
    for (int64_t i = 0; i < n; ++i) for (int z = 0; z < S; ++z)
        if (wr[(size_t)i * S + z] != 1) { printf("n=%ld body %ld slot %d written %d (R=%d D=%d kD=%d F=%d)\n", (long)n, (long)i, z, wr[(size_t)i * S + z], R, tl.D, tl.kD, tl.F); return 1; }
    if (verbose) printf("n=%ld tile(%d,%d) R=%d pairs=%ld F=%d D=%d kD=%d grid=%ld slots=%d (nb %d)\n", (long)n, tpl, waves, R, (long)U, tl.F, tl.D, tl.kD, (long)grid, S, nb);
    return 0;
}
int main()
{
    int bad = 0, cnt = 0;
    for (int64_t n : {1, 100, 4096, 5632, 8192, 9728, 9984, 10240, 10425, 11520, 13056, 16384, 23000, 30000, 40000, 46000, 46100, 131072}) bad |= check(n, 4, 4, true);
    for (int64_t n = 1; n <= 30000 && !bad; n += (n < 3000 ? 7 : 13)) { bad |= check(n, 4, 4, false); bad |= check(n, 2, 4, false); ++cnt; }
    printf("%s (%d sizes)\n", bad ? "FAIL" : "ok", cnt);
    return bad;
}
