// Autotuner of the stencil stage shape (the paper tunes its launch parameters
// per machine, Sec. "QUDA": threads per block, grid, shared memory).
//
// The tuned choice is the stencil form (register RHS tiles or LDS-staged links)
// and the number of RHS that share one link load, for a (lattice, precision,
// batch size) key.  Each candidate runs the two fused stages of the solver's
// M_hat on the solver's own workspace and is timed with HIP events; the
// fastest pair wins.  Choices live in the context for its lifetime and, when
// the environment variable LAPH_TUNE_CACHE names a file, are appended to that
// file and read back by later contexts of the same lattice, device
// architecture and stencil build.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "laph_solver.h"

namespace laph {

laph_status time_stage_pair(const Ctx &c, int prec, int nrhs, int form, int tile, int site_major, int mass_idx,
                            int reps, char *fields, double *partials, int *d_ints, double ms[2]) {
    const size_t hv = c.hv(prec);
    const int ntiles = (nrhs + tile - 1) / tile;
    std::vector<int> ints((size_t)ntiles * tile + ntiles + 1, -1);
    for (int r = 0; r < nrhs; ++r) ints[r] = r;
    for (int t = 0; t < ntiles; ++t) ints[(size_t)ntiles * tile + t] = mass_idx;
    ints.back() = ntiles;
    LAPH_HIP(hipMemcpyAsync(d_ints, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    // a fixed byte pattern (binary16 0x3c3c ~ 1.06, FP32 norms ~ 0.0115, FP32/FP64 values small)
    LAPH_HIP(hipMemsetAsync(fields, 0x3c, 4 * (size_t)nrhs * hv, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    Tiles t;
    t.slots = d_ints;
    t.mass = d_ints + (size_t)ntiles * tile;
    t.ntiles = d_ints + (size_t)ntiles * tile + ntiles;
    t.ntiles_max = ntiles;
    t.nr = tile;
    StageSpec s1;
    s1.prec = prec;
    s1.form = form;
    s1.site_major = site_major;
    s1.pstride = partial_stride(c);
    s1.out_parity = 1;
    s1.clover = 1;
    s1.in = Operand{fields, hv};
    s1.out = Operand{fields + (size_t)nrhs * hv, hv};
    s1.tiles = t;
    StageSpec s2 = s1;
    s2.out_parity = 0;
    s2.in = s1.out;
    s2.out = Operand{fields + 2 * (size_t)nrhs * hv, hv};
    s2.post = 1;
    s2.y = s1.in;
    s2.a = 1.0;
    s2.b = -0.25;
    s2.red = 1;
    s2.w = Operand{fields + 3 * (size_t)nrhs * hv, hv};
    s2.partials = partials;
    LAPH_TRY(launch_stage(c, s1));   // warm
    LAPH_TRY(launch_stage(c, s2));
    LAPH_HIP(hipEventRecord(c.ev[0], c.stream));
    for (int i = 0; i < reps; ++i) LAPH_TRY(launch_stage(c, s1));
    LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
    for (int i = 0; i < reps; ++i) LAPH_TRY(launch_stage(c, s2));
    LAPH_HIP(hipEventRecord(c.ev[2], c.stream));
    LAPH_HIP(hipEventSynchronize(c.ev[2]));
    float a = 0, b = 0;
    LAPH_HIP(hipEventElapsedTime(&a, c.ev[0], c.ev[1]));
    LAPH_HIP(hipEventElapsedTime(&b, c.ev[1], c.ev[2]));
    ms[0] = a / reps;
    ms[1] = b / reps;
    return LAPH_OK;
}

// candidates for a precision and batch size
static std::vector<Ctx::Shape> candidates(int prec, int nrhs) {
    std::vector<Ctx::Shape> out;
    for (int sm : {0, 1}) {
        for (int t : {1, 2, 4})
            if (t <= nrhs || t == 1) out.push_back({kFormRegister, t, sm});
        for (int t : {4, 8, 16})
            if (t <= nrhs || t == 4) out.push_back({kFormLds, t, sm});
    }
    return out;
}

static const char *cache_path() { return std::getenv("LAPH_TUNE_CACHE"); }

// Digest of the stencil sources this library was built from (set by the build
// script): a choice measured on other kernels is not reused.
#ifndef LAPH_STENCIL_DIGEST
#define LAPH_STENCIL_DIGEST "unversioned"
#endif
static const char *kCacheTag = "laph-tune-2";

// Cache lines: tag arch digest Lx Ly Lz Lt prec nrhs form tile site_major ms.
// The file is read whole; only lines of this lattice, architecture and
// stencil build are taken (a later line of the same key wins).
void load_tune_cache(Ctx &c) {
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    if (std::fseek(f, 0, SEEK_END) == 0) {
        const long n = std::ftell(f);
        if (n > 0 && std::fseek(f, 0, SEEK_SET) == 0) {
            text.resize((size_t)n);
            text.resize(std::fread(&text[0], 1, (size_t)n, f));
        }
    }
    std::fclose(f);
    size_t pos = 0;
    while (pos < text.size()) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) eol = text.size();
        const std::string line = text.substr(pos, eol - pos);
        pos = eol + 1;
        char tag[32], arch[64], digest[64];
        int d[4], prec, ns, form, tile, sm;
        double ms;
        if (std::sscanf(line.c_str(), "%31s %63s %63s %d %d %d %d %d %d %d %d %d %lf", tag, arch, digest, &d[0],
                        &d[1], &d[2], &d[3], &prec, &ns, &form, &tile, &sm, &ms) != 13)
            continue;
        if (std::strcmp(tag, kCacheTag) || std::strcmp(arch, c.arch) || std::strcmp(digest, LAPH_STENCIL_DIGEST))
            continue;
        if (d[0] == c.dims[0] && d[1] == c.dims[1] && d[2] == c.dims[2] && d[3] == c.dims[3])
            c.tuned[{prec, ns}] = Ctx::Shape{form, tile, sm};
    }
}

static void store_tune_cache(const Ctx &c, int prec, int ns, const Ctx::Shape &sh, double ms) {
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %s %s %d %d %d %d %d %d %d %d %d %.6f\n", kCacheTag, c.arch, LAPH_STENCIL_DIGEST, c.dims[0],
                 c.dims[1], c.dims[2], c.dims[3], prec, ns, sh.form, sh.tile, sh.site_major, ms);
    std::fclose(f);
}

laph_status autotune_stencil(Ctx &c, int prec, int nrhs, int mass_idx, char *fields, double *partials, int *d_ints,
                             Ctx::Shape *out, double *ms_out) {
    double best = 1e300;
    Ctx::Shape bsh{kFormRegister, 1, 0};
    for (const auto &cand : candidates(prec, nrhs)) {
        double ms[2];
        LAPH_TRY(time_stage_pair(c, prec, nrhs, cand.form, cand.tile, cand.site_major, mass_idx, 3, fields, partials,
                                 d_ints, ms));
        if (ms[0] + ms[1] < best) {
            best = ms[0] + ms[1];
            bsh = cand;
        }
    }
    c.tuned[{prec, nrhs}] = bsh;
    store_tune_cache(c, prec, nrhs, bsh, best);
    *out = bsh;
    if (ms_out) *ms_out = best;
    return LAPH_OK;
}

size_t tune_ints(int nrhs) { return (size_t)nrhs * 16 + (size_t)nrhs + 8; }

}  // namespace laph
