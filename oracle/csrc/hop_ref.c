/*
 * Oracle (test infrastructure only): plain reference of the Wilson hopping term
 *
 *   (H psi)(x) = sum_mu [ eta+ (1 - g*gamma_mu) U_mu(x) psi(x+mu)
 *                        + eta- (1 + g*gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]
 *
 * with g = +1 (H) or g = -1 (gamma5 H gamma5, "dagger"), eta = -1 on hops that
 * cross the time boundary when the time direction is antiperiodic, +1 otherwise.
 * The quark propagator is the inverse of the Dirac matrix applied to a source
 * (paper, Sec. "Current state-of-the-art"); the Wilson-clover form used here
 * and its conventions are this project's reading of the unspecified operator.
 *
 * Straight site loop, full 4x4 spin matrices (no spin projection), FP64 complex.
 * Layouts (C order, interleaved complex):
 *   U   [t][z][y][x][mu][a][b]          mu = 0..3 <-> x,y,z,t
 *   psi [r][t][z][y][x][s][a]           r = right-hand side
 *   gam [mu][s][s']                     the four gamma matrices, supplied by the caller
 * Only tests, the smoke check and the CPU baseline leg of the benchmark use it.
 */
#include <complex.h>
#include <stddef.h>

typedef double complex cplx;

void oracle_hop(const cplx *U, const cplx *psi, cplx *out, const cplx *gam,
                int lx, int ly, int lz, int lt, int nrhs, int antiperiodic_t,
                int dagger)
{
    const long vol = (long)lx * ly * lz * lt;
    const int ext[4] = {lx, ly, lz, lt};
    const double g = dagger ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (long rs = 0; rs < (long)nrhs * vol; ++rs) {
        const long r = rs / vol;
        const long i = rs % vol;
        int c[4];
        c[0] = (int)(i % lx);
        c[1] = (int)((i / lx) % ly);
        c[2] = (int)((i / ((long)lx * ly)) % lz);
        c[3] = (int)(i / ((long)lx * ly * lz));
        cplx acc[4][3];
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) acc[s][a] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                /* dir 0: forward neighbour x+mu, link U_mu(x);
                   dir 1: backward neighbour x-mu, link U_mu(x-mu)^dagger */
                int n[4] = {c[0], c[1], c[2], c[3]};
                double eta = 1.0;
                if (dir == 0) {
                    n[mu] = c[mu] + 1;
                    if (n[mu] == ext[mu]) {
                        n[mu] = 0;
                        if (mu == 3 && antiperiodic_t) eta = -1.0;
                    }
                } else {
                    n[mu] = c[mu] - 1;
                    if (n[mu] < 0) {
                        n[mu] = ext[mu] - 1;
                        if (mu == 3 && antiperiodic_t) eta = -1.0;
                    }
                }
                const long j = n[0] + (long)lx * (n[1] + (long)ly * (n[2] + (long)lz * n[3]));
                const cplx *link = U + ((dir == 0 ? i : j) * 4 + mu) * 9;
                const cplx *src = psi + (r * vol + j) * 12;
                /* W = link (or its adjoint) acting on colour, all four spins */
                cplx w[4][3];
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx sum = 0;
                        for (int b = 0; b < 3; ++b) {
                            cplx m = (dir == 0) ? link[a * 3 + b] : conj(link[b * 3 + a]);
                            sum += m * src[s * 3 + b];
                        }
                        w[s][a] = eta * sum;
                    }
                /* (1 -/+ g gamma_mu) on spin */
                const double sg = (dir == 0) ? -g : g;
                const cplx *gm = gam + mu * 16;
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx sum = w[s][a];
                        for (int t = 0; t < 4; ++t) sum += sg * gm[s * 4 + t] * w[t][a];
                        acc[s][a] += sum;
                    }
            }
        }
        cplx *dst = out + (r * vol + i) * 12;
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) dst[s * 3 + a] = acc[s][a];
    }
}
