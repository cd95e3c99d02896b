/*
 * cpu_cells.c -- CPU baseline of the dynamic cutoff method's force step as
 * the paper runs it on CPU clusters: linked cells with small bins, a
 * per-step neighbour list (Algorithm 2.2) and the dynamic-cutoff force loop
 * over it (Algorithm 2.3), both parallelised with OpenMP dynamic scheduling
 * in chunks of 20 particles (Section 2.4).  FP64, Lennard-Jones 12-6,
 * own-cutoff rule (j acts on i iff r_ij < r_c(i)), no Newton's third law.
 *
 * TEST INFRASTRUCTURE ONLY: it gives the benchmark a CPU throughput figure to
 * set beside the GPU's, and the tests check it against the O(N^2) oracle.  It
 * is not the parity authority and shares no code with the HIP library.
 *
 * Bins have edge >= r_c^min + r_s (the "small bins" of Section 2.3: the
 * smallest cutoff plus the skin, instead of the largest), and a particle
 * scans as many bins in each direction as its own cutoff needs.  The skin
 * r_s is 0: the list is rebuilt for every force evaluation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double now_s(void) {
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

static int64_t wrapi(int64_t a, int64_t n) {
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/*
 * Forces on the particles idx[0..nidx) (all n when idx is NULL) from all n
 * particles.  Outputs per listed particle: fx, fy, fz, nnbr; *energy = half
 * the sum of their pair energies.  Returns the interacting ordered pairs.
 * t_build / t_force receive the seconds of the list build and of the force
 * loop.  Returns -1 if memory runs out.
 */
int64_t cpu_cells_forces(int64_t n, const double *x, const double *y, const double *z,
                         const double *rc, const double *L, double bin_edge, double eps,
                         double sigma, const int64_t *idx, int64_t nidx, double *fx,
                         double *fy, double *fz, int32_t *nnbr, double *energy, double *t_build,
                         double *t_force) {
    if (!idx) nidx = n;
    int64_t nb[3], nbins = 1;
    for (int a = 0; a < 3; ++a) {
        nb[a] = (int64_t)floor(L[a] / bin_edge);
        if (nb[a] < 1) nb[a] = 1;
        nbins *= nb[a];
    }
    double bl[3] = {L[0] / nb[0], L[1] / nb[1], L[2] / nb[2]};
    /* binning: counting sort of particle indices by bin */
    int64_t *head = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    int64_t *bin_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *members = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
    int64_t *lstart = (int64_t *)malloc((size_t)(nidx + 1) * sizeof(int64_t));
    if (!head || !bin_of || !members || !fill || !lstart) {
        free(head); free(bin_of); free(members); free(fill); free(lstart);
        return -1;
    }
    double t0 = now_s();
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        double p[3] = {x[i], y[i], z[i]};
        for (int a = 0; a < 3; ++a) {
            double w = p[a] - L[a] * floor(p[a] / L[a]);
            c[a] = (int64_t)floor(w / bl[a]);
            if (c[a] >= nb[a]) c[a] = nb[a] - 1;
            if (c[a] < 0) c[a] = 0;
        }
        bin_of[i] = (c[2] * nb[1] + c[1]) * nb[0] + c[0];
        head[bin_of[i] + 1] += 1;
    }
    for (int64_t b = 0; b < nbins; ++b) head[b + 1] += head[b];
    for (int64_t i = 0; i < n; ++i) members[head[bin_of[i]] + fill[bin_of[i]]++] = i;

    /* Algorithm 2.2: per particle, the j within r_c(i) + r_s (r_s = 0),
     * found in the bins its cutoff reaches; first count, then fill */
    int64_t *count = (int64_t *)calloc((size_t)(nidx > 0 ? nidx : 1), sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *list = NULL;
        if (pass == 1) {
            lstart[0] = 0;
            for (int64_t q = 0; q < nidx; ++q) lstart[q + 1] = lstart[q] + count[q];
            list = (int64_t *)malloc((size_t)(lstart[nidx] > 0 ? lstart[nidx] : 1) *
                                     sizeof(int64_t));
            if (!list) {
                free(head); free(bin_of); free(members); free(fill); free(lstart); free(count);
                return -1;
            }
        }
#pragma omp parallel for schedule(dynamic, 20)
        for (int64_t q = 0; q < nidx; ++q) {
            const int64_t i = idx ? idx[q] : q;
            const double xi = x[i], yi = y[i], zi = z[i], R = rc[i], R2 = R * R;
            const int64_t b = bin_of[i];
            const int64_t cx = b % nb[0], cy = (b / nb[0]) % nb[1], cz = b / (nb[0] * nb[1]);
            /* bins within reach along each axis; every bin once when the
             * reach wraps all the way round */
            int64_t lo[3], hi[3];
            int full[3];
            const int64_t c3[3] = {cx, cy, cz};
            for (int a = 0; a < 3; ++a) {
                const int64_t reach = (int64_t)ceil(R / bl[a]);
                full[a] = 2 * reach + 1 >= nb[a];
                if (full[a]) {
                    lo[a] = 0;
                    hi[a] = nb[a] - 1;
                } else {
                    lo[a] = c3[a] - reach;
                    hi[a] = c3[a] + reach;
                }
            }
            /* distance from the particle to the near face of a bin b
             * bins away along axis a (0 for its own bin): bins beyond the
             * cutoff sphere are skipped, as a LAMMPS bin stencil does */
            double off[3];
            const double p3[3] = {xi - L[0] * floor(xi / L[0]), yi - L[1] * floor(yi / L[1]),
                                  zi - L[2] * floor(zi / L[2])};
            for (int a = 0; a < 3; ++a) off[a] = p3[a] - (double)c3[a] * bl[a];
#define GAP(a, bcell)                                                                    \
    (full[a] ? 0.0                                                                       \
             : ((bcell) > c3[a] ? (double)((bcell) - c3[a] - 1) * bl[a] + (bl[a] - off[a]) \
                : ((bcell) < c3[a] ? (double)(c3[a] - (bcell) - 1) * bl[a] + off[a] : 0.0)))
            int64_t k = 0;
            for (int64_t bz = lo[2]; bz <= hi[2]; ++bz) {
                const double gz = GAP(2, bz);
                if (gz * gz >= R2) continue;
                for (int64_t by = lo[1]; by <= hi[1]; ++by) {
                    const double gy = GAP(1, by);
                    if (gz * gz + gy * gy >= R2) continue;
                    for (int64_t bx = lo[0]; bx <= hi[0]; ++bx) {
                        const double gx = GAP(0, bx);
                        if (gz * gz + gy * gy + gx * gx >= R2) continue;
                        const int64_t bb =
                            (wrapi(bz, nb[2]) * nb[1] + wrapi(by, nb[1])) * nb[0] + wrapi(bx, nb[0]);
                        /* the periodic image a bin beyond the box edge holds
                         * (LAMMPS-style ghosts); an axis whose reach wraps the
                         * whole box takes the minimum image instead */
                        const double sx = full[0] ? 0.0 : (bx < 0 ? -L[0] : (bx >= nb[0] ? L[0] : 0.0));
                        const double sy = full[1] ? 0.0 : (by < 0 ? -L[1] : (by >= nb[1] ? L[1] : 0.0));
                        const double sz = full[2] ? 0.0 : (bz < 0 ? -L[2] : (bz >= nb[2] ? L[2] : 0.0));
                        for (int64_t m = head[bb]; m < head[bb + 1]; ++m) {
                            const int64_t j = members[m];
                            if (j == i) continue;
                            double ddx = xi - (x[j] + sx), ddy = yi - (y[j] + sy),
                                   ddz = zi - (z[j] + sz);
                            if (full[0]) ddx -= L[0] * rint(ddx / L[0]);
                            if (full[1]) ddy -= L[1] * rint(ddy / L[1]);
                            if (full[2]) ddz -= L[2] * rint(ddz / L[2]);
                            const double r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
                            if (r2 < R2) {
                                if (pass == 1) list[lstart[q] + k] = j;
                                ++k;
                            }
                        }
                    }
                }
            }
#undef GAP
            if (pass == 0) count[q] = k;
        }
        if (pass == 1) {
            double t1 = now_s();
            /* Algorithm 2.3: forces from the list, j acting on i iff r_ij < r_c(i) */
            double esum = 0.0;
            const double sig2 = sigma * sigma;
#pragma omp parallel for schedule(dynamic, 20) reduction(+ : esum)
            for (int64_t q = 0; q < nidx; ++q) {
                const int64_t i = idx ? idx[q] : q;
                const double xi = x[i], yi = y[i], zi = z[i], R2 = rc[i] * rc[i];
                double Fx = 0.0, Fy = 0.0, Fz = 0.0, e = 0.0;
                int32_t cnt = 0;
                for (int64_t m = lstart[q]; m < lstart[q + 1]; ++m) {
                    const int64_t j = list[m];
                    double ddx = xi - x[j], ddy = yi - y[j], ddz = zi - z[j];
                    ddx -= L[0] * rint(ddx / L[0]);
                    ddy -= L[1] * rint(ddy / L[1]);
                    ddz -= L[2] * rint(ddz / L[2]);
                    const double r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
                    if (!(r2 < R2)) continue;
                    const double r2i = 1.0 / r2;
                    const double s2 = sig2 * r2i;
                    const double s6 = s2 * s2 * s2;
                    const double fpair = 24.0 * eps * s6 * (2.0 * s6 - 1.0) * r2i;
                    Fx += fpair * ddx;
                    Fy += fpair * ddy;
                    Fz += fpair * ddz;
                    e += 2.0 * eps * s6 * (s6 - 1.0);
                    ++cnt;
                }
                fx[q] = Fx;
                fy[q] = Fy;
                fz[q] = Fz;
                if (nnbr) nnbr[q] = cnt;
                esum += e;
            }
            double t2 = now_s();
            if (t_build) *t_build = t1 - t0;
            if (t_force) *t_force = t2 - t1;
            if (energy) *energy = esum;
            free(list);
        }
    }
    int64_t pairs = 0;
    if (nnbr)
        for (int64_t q = 0; q < nidx; ++q) pairs += nnbr[q];
    free(head); free(bin_of); free(members); free(fill); free(lstart); free(count);
    return pairs;
}
