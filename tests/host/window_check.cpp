// Host-side check of the site-window helpers (compiled by the test with hipcc; runs
// on the CPU).  Reads "vh lo n h0 cnt" lines and prints, per line, in_window(h0) and
// block_outside(h0, cnt); reads "geom lx ly lz lt t0 k" lines and prints slab_window.
#include <cstdio>
#include <cstring>

#include "../../paper_2510_26313_amd/csrc/laph_internal.h"

int main() {
    char tag[16];
    while (std::scanf("%15s", tag) == 1) {
        if (!std::strcmp(tag, "win")) {
            int vh, lo, n, h0, cnt;
            if (std::scanf("%d %d %d %d %d", &vh, &lo, &n, &h0, &cnt) != 5) return 1;
            laph::SiteWindow w;
            w.lo = lo;
            w.n = n;
            std::printf("%d %d\n", laph::in_window(w, h0, vh) ? 1 : 0, laph::block_outside(w, h0, cnt, vh) ? 1 : 0);
        } else if (!std::strcmp(tag, "slab")) {
            int lx, ly, lz, lt, t0, k;
            if (std::scanf("%d %d %d %d %d %d", &lx, &ly, &lz, &lt, &t0, &k) != 6) return 1;
            laph::Geom g{};
            g.lx = lx;
            g.ly = ly;
            g.lz = lz;
            g.lt = lt;
            g.lxh = lx / 2;
            g.vs_h = lx * ly * lz / 2;
            g.vh = g.vs_h * lt;
            const laph::SiteWindow w = laph::slab_window(g, t0, k);
            std::printf("%d %d\n", w.lo, w.n);
        } else {
            return 1;
        }
    }
    return 0;
}
