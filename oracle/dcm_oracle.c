/*
 * dcm_oracle.c -- plain, slow FP64 CPU oracle for the dynamic cutoff method
 * (Springer, Ismail, Bientinesi, "A Scalable, Linear-Time Dynamic Cutoff
 * Algorithm for Molecular Dynamics").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Every step is written in its plainest serial form, in FP64, compiled with
 * -ffp-contract=off so that no multiply-add is fused behind our back, and
 * every long sum uses Neumaier-compensated accumulation.
 *
 * Readings of points the paper leaves open are marked "reading:" and are the
 * same ones the design notes list.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated accumulator                                          */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static inline double ks_val(const ksum *k) { return k->s + k->c; }

static inline int64_t imod(int64_t a, int64_t n) {
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Step 1: periodic wrap (the domain is periodic, Section 2 "parallelization")*/
/* w = x - L*floor(x/L); a result that rounds to L (or below 0) is folded.   */
/* ------------------------------------------------------------------------ */
static inline double wrap1(double x, double L) {
    double q = floor(x / L);
    double w = x - L * q;
    if (w < 0.0) w = w + L;
    if (w >= L) w = 0.0;
    return w;
}

void orc_wrap(int64_t n, double *x, double *y, double *z, const double *L) {
    for (int64_t i = 0; i < n; ++i) {
        x[i] = wrap1(x[i], L[0]);
        y[i] = wrap1(y[i], L[1]);
        z[i] = wrap1(z[i], L[2]);
    }
}

/* ------------------------------------------------------------------------ */
/* Grid geometry (Section 2.1, footnote 2: the voxel edge h is chosen once). */
/* reading: N_a = max(1, round(L_a/h)), h_a = L_a/N_a (anisotropic voxels).  */
/* ------------------------------------------------------------------------ */
void orc_grid_dims(const double *L, double h, int32_t *nv, double *hv) {
    for (int a = 0; a < 3; ++a) {
        double r = round(L[a] / h);
        int32_t k = (int32_t)r;
        if (k < 1) k = 1;
        nv[a] = k;
        hv[a] = L[a] / (double)k;
    }
}

static inline int32_t cell_index_1d(double x, double scale, int32_t n) {
    /* x is already wrapped into [0, L); scale = n/L computed once */
    int32_t c = (int32_t)floor(x * scale);
    if (c > n - 1) c = n - 1;
    if (c < 0) c = 0;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Step 2: bin particles into h x h x h boxes (Section 2.1, Fig. 4a).        */
/* ------------------------------------------------------------------------ */
void orc_voxel_counts(int64_t n, const double *x, const double *y, const double *z,
                      const double *L, const int32_t *nv, uint32_t *counts) {
    int64_t nvox = (int64_t)nv[0] * nv[1] * nv[2];
    double sx = (double)nv[0] / L[0], sy = (double)nv[1] / L[1], sz = (double)nv[2] / L[2];
    memset(counts, 0, (size_t)nvox * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        double wx = wrap1(x[i], L[0]), wy = wrap1(y[i], L[1]), wz = wrap1(z[i], L[2]);
        int64_t vx = cell_index_1d(wx, sx, nv[0]);
        int64_t vy = cell_index_1d(wy, sy, nv[1]);
        int64_t vz = cell_index_1d(wz, sz, nv[2]);
        counts[(vz * nv[1] + vy) * nv[0] + vx] += 1u;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3: gray value = relative particle density of each voxel (Fig. 4b).   */
/* reading: the sum of counts over the periodic 3x3x3 window (an integer;    */
/* a common scale factor does not move a threshold).                         */
/* ------------------------------------------------------------------------ */
void orc_gray27(const int32_t *nv, const uint32_t *counts, uint32_t *g) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2];
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                uint32_t s = 0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx)
                            s += counts[(imod(k + dz, nz) * ny + imod(j + dy, ny)) * nx +
                                        imod(i + dx, nx)];
                g[(k * ny + j) * nx + i] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* Step 4a: two-phase piecewise-constant segmentation, data term only        */
/* (Section 2.1; Mumford-Shah with no length penalty is the 2-means split).  */
/* For a threshold t the phases are {g >= t} and {g < t}; the best t         */
/* maximises S0^2/n0 + S1^2/n1 (equivalently minimises the within-class sum  */
/* of squares).  Ties go to the smallest t.  Sums are exact integers,        */
/* converted to double, and combined in exactly this order.                  */
/* Returns 0, or 1 if the volume holds a single phase (every g equal, or a   */
/* density contrast (c1+3)/(c0+3) below 2).                                  */
/* ------------------------------------------------------------------------ */
int orc_otsu(int64_t nvox, const uint32_t *g, int32_t *t_out, double *c0_out, double *c1_out) {
    uint32_t gmax = 0;
    for (int64_t v = 0; v < nvox; ++v) if (g[v] > gmax) gmax = g[v];
    int64_t *hist = (int64_t *)calloc((size_t)gmax + 2, sizeof(int64_t));
    for (int64_t v = 0; v < nvox; ++v) hist[g[v]] += 1;
    int64_t total_n = nvox, total_s = 0;
    for (int64_t t = 0; t <= (int64_t)gmax; ++t) total_s += hist[t] * t;
    /* n1, S1: count and sum of g >= t, built from the top down */
    double best = -1.0;
    int32_t best_t = -1;
    int64_t n1 = 0, s1 = 0;
    int64_t *n1_at = (int64_t *)calloc((size_t)gmax + 2, sizeof(int64_t));
    int64_t *s1_at = (int64_t *)calloc((size_t)gmax + 2, sizeof(int64_t));
    for (int64_t t = (int64_t)gmax; t >= 0; --t) {
        n1 += hist[t];
        s1 += hist[t] * t;
        n1_at[t] = n1;
        s1_at[t] = s1;
    }
    for (int64_t t = 1; t <= (int64_t)gmax; ++t) {
        int64_t nn1 = n1_at[t], ss1 = s1_at[t];
        int64_t nn0 = total_n - nn1, ss0 = total_s - ss1;
        if (nn0 == 0 || nn1 == 0) continue;
        double S0 = (double)ss0, S1 = (double)ss1;
        double score = (S0 * S0) / (double)nn0 + (S1 * S1) / (double)nn1;
        if (score > best) { best = score; best_t = (int32_t)t; }
    }
    int degenerate = 0;
    double c0 = 0.0, c1 = 0.0;
    if (best_t < 0) {
        degenerate = 1;
    } else {
        int64_t nn1 = n1_at[best_t], ss1 = s1_at[best_t];
        int64_t nn0 = total_n - nn1, ss0 = total_s - ss1;
        c0 = (double)ss0 / (double)nn0;
        c1 = (double)ss1 / (double)nn1;
        if ((c1 + 3.0) / (c0 + 3.0) < 2.0) degenerate = 1;
    }
    free(hist); free(n1_at); free(s1_at);
    *t_out = best_t;
    if (c0_out) *c0_out = c0;
    if (c1_out) *c1_out = c1;
    return degenerate;
}

/* ------------------------------------------------------------------------ */
/* Step 4b: regularise the phase map.  reading: stand-in for the length term */
/* of the Mumford-Shah functional -- a synchronous 27-neighbour majority     */
/* vote, s <- [sum of s over the periodic 3x3x3 window >= 14], repeated      */
/* until nothing changes, until a pass reproduces the state of two passes    */
/* ago (a 2-cycle; the current state is kept), or for at most max_passes.    */
/* Returns the number of passes run.                                         */
/* ------------------------------------------------------------------------ */
int orc_majority(const int32_t *nv, uint8_t *s, int max_passes) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2], nvox = nx * ny * nz;
    uint8_t *prev = (uint8_t *)malloc((size_t)nvox);  /* state one pass ago   */
    uint8_t *prev2 = (uint8_t *)malloc((size_t)nvox); /* state two passes ago */
    uint8_t *next = (uint8_t *)malloc((size_t)nvox);
    memcpy(prev, s, (size_t)nvox);
    int have_prev2 = 0, passes = 0;
    while (passes < max_passes) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int sum = 0;
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx)
                                sum += prev[(imod(k + dz, nz) * ny + imod(j + dy, ny)) * nx +
                                            imod(i + dx, nx)];
                    next[(k * ny + j) * nx + i] = (uint8_t)(sum >= 14 ? 1 : 0);
                }
        ++passes;
        int same_as_prev = memcmp(next, prev, (size_t)nvox) == 0;
        int same_as_prev2 = have_prev2 && memcmp(next, prev2, (size_t)nvox) == 0;
        memcpy(prev2, prev, (size_t)nvox);
        have_prev2 = 1;
        memcpy(prev, next, (size_t)nvox);
        if (same_as_prev || same_as_prev2) break;
    }
    memcpy(s, prev, (size_t)nvox);
    free(prev); free(prev2); free(next);
    return passes;
}

/* ------------------------------------------------------------------------ */
/* Step 4b': regularise with the length term of the two-phase piecewise-     */
/* constant Mumford-Shah energy (Section 2.1).  reading: on the voxel grid   */
/* the energy is sum_v (g_v - c_{s_v})^2 + nu * (number of periodic 26-      */
/* neighbour pairs in different phases), minimised over s by synchronous     */
/* iterated conditional modes with the phase means c0, c1 of the two-phase   */
/* split held fixed.  A pass sets each voxel to the phase of lower local     */
/* energy: d = ((g - c1)^2 - (g - c0)^2) + nu * (26 - 2 n1), with n1 its     */
/* 26 neighbours in phase 1; s = 1 if d < 0, 0 if d > 0, unchanged if d = 0. */
/* The passes stop as the majority vote's do (fixed point, 2-cycle or        */
/* max_passes).  Returns the number of passes run.                           */
/* ------------------------------------------------------------------------ */
int orc_potts(const int32_t *nv, const uint32_t *g, double c0, double c1, double nu, uint8_t *s,
              int max_passes) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2], nvox = nx * ny * nz;
    uint8_t *prev = (uint8_t *)malloc((size_t)nvox);
    uint8_t *prev2 = (uint8_t *)malloc((size_t)nvox);
    uint8_t *next = (uint8_t *)malloc((size_t)nvox);
    memcpy(prev, s, (size_t)nvox);
    int have_prev2 = 0, passes = 0;
    while (passes < max_passes) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t v = (k * ny + j) * nx + i;
                    int n1 = 0;
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx)
                                if (dx || dy || dz)
                                    n1 += prev[(imod(k + dz, nz) * ny + imod(j + dy, ny)) * nx +
                                               imod(i + dx, nx)];
                    double a = (double)g[v] - c1, b = (double)g[v] - c0;
                    double d = (a * a - b * b) + nu * (double)(26 - 2 * n1);
                    next[v] = d < 0.0 ? 1 : (d > 0.0 ? 0 : prev[v]);
                }
        ++passes;
        int same_as_prev = memcmp(next, prev, (size_t)nvox) == 0;
        int same_as_prev2 = have_prev2 && memcmp(next, prev2, (size_t)nvox) == 0;
        memcpy(prev2, prev, (size_t)nvox);
        have_prev2 = 1;
        memcpy(prev, next, (size_t)nvox);
        if (same_as_prev || same_as_prev2) break;
    }
    memcpy(s, prev, (size_t)nvox);
    free(prev); free(prev2); free(next);
    return passes;
}

/* ------------------------------------------------------------------------ */
/* Step 4c: bubble filter (Section 2.1): connected components of either      */
/* phase smaller than a user-given volume are removed.  reading: components  */
/* are 6-connected with periodic neighbours, volumes count voxels, and every */
/* component with fewer than min_volume voxels takes the other phase, all on */
/* the same input map.  label[v] (may be NULL) gets the smallest voxel index */
/* of v's component.  Breadth-first search.  Returns the number of voxels    */
/* flipped.                                                                  */
/* ------------------------------------------------------------------------ */
int64_t orc_bubble_filter(const int32_t *nv, uint8_t *s, int64_t min_volume, int32_t *label) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2], nvox = nx * ny * nz;
    int32_t *lab = (int32_t *)malloc((size_t)nvox * sizeof(int32_t));
    int64_t *queue = (int64_t *)malloc((size_t)nvox * sizeof(int64_t));
    uint8_t *flip = (uint8_t *)calloc((size_t)nvox, 1);
    for (int64_t v = 0; v < nvox; ++v) lab[v] = -1;
    for (int64_t start = 0; start < nvox; ++start) {
        if (lab[start] >= 0) continue;
        /* visiting voxels in increasing order: start is the component's smallest index */
        int64_t head = 0, tail = 0;
        queue[tail++] = start;
        lab[start] = (int32_t)start;
        while (head < tail) {
            int64_t v = queue[head++];
            int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
            int64_t nb[6] = {(k * ny + j) * nx + imod(i - 1, nx), (k * ny + j) * nx + imod(i + 1, nx),
                             (k * ny + imod(j - 1, ny)) * nx + i, (k * ny + imod(j + 1, ny)) * nx + i,
                             (imod(k - 1, nz) * ny + j) * nx + i, (imod(k + 1, nz) * ny + j) * nx + i};
            for (int q = 0; q < 6; ++q) {
                int64_t u = nb[q];
                if (lab[u] < 0 && s[u] == s[v]) {
                    lab[u] = (int32_t)start;
                    queue[tail++] = u;
                }
            }
        }
        if (tail < min_volume)
            for (int64_t q = 0; q < tail; ++q) flip[queue[q]] = 1;
    }
    int64_t flipped = 0;
    for (int64_t v = 0; v < nvox; ++v)
        if (flip[v]) { s[v] = (uint8_t)(1 - s[v]); ++flipped; }
    if (label) memcpy(label, lab, (size_t)nvox * sizeof(int32_t));
    free(lab); free(queue); free(flip);
    return flipped;
}

/* ------------------------------------------------------------------------ */
/* Step 5: the interface is where adjacent boxes carry different phases      */
/* (Section 2.1, Fig. 4c).  reading: a voxel is an interface voxel when it   */
/* is high-density and one of its 6 periodic face neighbours is low-density. */
/* ------------------------------------------------------------------------ */
void orc_interface(const int32_t *nv, const uint8_t *s, uint8_t *iface) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2];
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t v = (k * ny + j) * nx + i;
                uint8_t f = 0;
                if (s[v]) {
                    if (!s[(k * ny + j) * nx + imod(i - 1, nx)]) f = 1;
                    if (!s[(k * ny + j) * nx + imod(i + 1, nx)]) f = 1;
                    if (!s[(k * ny + imod(j - 1, ny)) * nx + i]) f = 1;
                    if (!s[(k * ny + imod(j + 1, ny)) * nx + i]) f = 1;
                    if (!s[(imod(k - 1, nz) * ny + j) * nx + i]) f = 1;
                    if (!s[(imod(k + 1, nz) * ny + j) * nx + i]) f = 1;
                }
                iface[v] = f;
            }
}

/* ------------------------------------------------------------------------ */
/* Step 6: box-interface distances (Section 2.2, Algorithm 2.1).             */
/* The local distance solve is the first-order Godunov upwind update of the  */
/* eikonal equation |grad d| = 1 used by the fast sweeping method: with the  */
/* smaller face neighbour a_k along each axis and spacing h_k, d solves      */
/*   sum over the m smallest a_k of ((d - a_k)/h_k)^2 = 1,                    */
/* taking the largest m whose root does not exceed the next a_k.             */
/* Written relative to the smallest a (e = d - a_min) to avoid cancellation. */
/* ------------------------------------------------------------------------ */
double orc_godunov(double ax, double ay, double az, double hx, double hy, double hz) {
    double a[3] = {ax, ay, az}, h[3] = {hx, hy, hz};
    /* sort (a, h) ascending by a; equal a keep axis order */
    for (int p = 1; p < 3; ++p)
        for (int q = p; q > 0 && a[q] < a[q - 1]; --q) {
            double ta = a[q]; a[q] = a[q - 1]; a[q - 1] = ta;
            double th = h[q]; h[q] = h[q - 1]; h[q - 1] = th;
        }
    if (isinf(a[0])) return INFINITY;
    double d = a[0] + h[0];
    if (d <= a[1]) return d;
    /* two terms: w0 e^2 + w1 (e - b1)^2 = 1 */
    double w0 = 1.0 / (h[0] * h[0]), w1 = 1.0 / (h[1] * h[1]);
    double b1 = a[1] - a[0];
    double A = w0 + w1;
    double B = w1 * b1;
    double C = w1 * b1 * b1 - 1.0;
    double disc = B * B - A * C;
    if (disc < 0.0) disc = 0.0;
    d = a[0] + (B + sqrt(disc)) / A;
    if (d <= a[2]) return d;
    /* three terms */
    double w2 = 1.0 / (h[2] * h[2]);
    double b2 = a[2] - a[0];
    A = (w0 + w1) + w2;
    B = w1 * b1 + w2 * b2;
    C = (w1 * b1 * b1 + w2 * b2 * b2) - 1.0;
    disc = B * B - A * C;
    if (disc < 0.0) disc = 0.0;
    return a[0] + (B + sqrt(disc)) / A;
}

/* Initialise D (Algorithm 2.1: interface and low-density boxes start at 0,  */
/* high-density boxes at +infinity), then run Gauss-Seidel sweeps in the 8   */
/* alternating axis orderings of the fast sweeping method.  As in Algorithm  */
/* 2.1, a new value is only accepted when it does not exceed rc_grid.        */
/* reading: the stopping threshold is exact -- stop after a full 8-ordering  */
/* pass that changes nothing.  Finally D <- min(D, rc_grid).                 */
/* Returns the number of full passes, or -1 if max_passes did not converge.  */
int orc_fsm(const int32_t *nv, const double *hv, const uint8_t *s, const uint8_t *iface,
            double rc_grid, int max_passes, double *D) {
    int64_t nx = nv[0], ny = nv[1], nz = nv[2], nvox = nx * ny * nz;
    for (int64_t v = 0; v < nvox; ++v) D[v] = (s[v] == 0 || iface[v]) ? 0.0 : INFINITY;
    int passes = 0, converged = 0;
    while (passes < max_passes) {
        int changed = 0;
        for (int o = 0; o < 8; ++o) {
            int sx = (o & 1) ? -1 : 1, sy = (o & 2) ? -1 : 1, sz = (o & 4) ? -1 : 1;
            for (int64_t kk = 0; kk < nz; ++kk) {
                int64_t k = sz > 0 ? kk : nz - 1 - kk;
                for (int64_t jj = 0; jj < ny; ++jj) {
                    int64_t j = sy > 0 ? jj : ny - 1 - jj;
                    for (int64_t ii = 0; ii < nx; ++ii) {
                        int64_t i = sx > 0 ? ii : nx - 1 - ii;
                        int64_t v = (k * ny + j) * nx + i;
                        if (s[v] == 0 || iface[v]) continue;
                        double axm = D[(k * ny + j) * nx + imod(i - 1, nx)];
                        double axp = D[(k * ny + j) * nx + imod(i + 1, nx)];
                        double aym = D[(k * ny + imod(j - 1, ny)) * nx + i];
                        double ayp = D[(k * ny + imod(j + 1, ny)) * nx + i];
                        double azm = D[(imod(k - 1, nz) * ny + j) * nx + i];
                        double azp = D[(imod(k + 1, nz) * ny + j) * nx + i];
                        double g = orc_godunov(fmin(axm, axp), fmin(aym, ayp), fmin(azm, azp),
                                               hv[0], hv[1], hv[2]);
                        if (g < D[v] && g <= rc_grid) { D[v] = g; changed = 1; }
                    }
                }
            }
        }
        ++passes;
        if (!changed) { converged = 1; break; }
    }
    for (int64_t v = 0; v < nvox; ++v) if (D[v] > rc_grid) D[v] = rc_grid;
    return converged ? passes : -1;
}

/* ------------------------------------------------------------------------ */
/* Steps 7-8: particle-interface distance by trilinear interpolation of the  */
/* voxel-centred D (Section 2.2), and the cutoff as a function of it.        */
/* reading: periodic interpolation between voxel centres; the cutoff ramps   */
/* linearly from rc_max at the interface down to rc_min at distance >= ramp. */
/* ------------------------------------------------------------------------ */
void orc_particle_distance(int64_t n, const double *x, const double *y, const double *z,
                           const double *L, const int32_t *nv, const double *D, double *delta) {
    double sc[3] = {(double)nv[0] / L[0], (double)nv[1] / L[1], (double)nv[2] / L[2]};
    int64_t nx = nv[0], ny = nv[1];
    for (int64_t p = 0; p < n; ++p) {
        double pos[3] = {wrap1(x[p], L[0]), wrap1(y[p], L[1]), wrap1(z[p], L[2])};
        int64_t i0[3], i1[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double u = pos[a] * sc[a] - 0.5;
            double f = floor(u);
            t[a] = u - f;
            int64_t ia = (int64_t)f;
            i0[a] = imod(ia, nv[a]);
            i1[a] = imod(ia + 1, nv[a]);
        }
#define DV(I, J, K) D[((K) * ny + (J)) * nx + (I)]
        double wx0 = 1.0 - t[0], wx1 = t[0];
        double wy0 = 1.0 - t[1], wy1 = t[1];
        double wz0 = 1.0 - t[2], wz1 = t[2];
        double c00 = DV(i0[0], i0[1], i0[2]) * wx0 + DV(i1[0], i0[1], i0[2]) * wx1;
        double c10 = DV(i0[0], i1[1], i0[2]) * wx0 + DV(i1[0], i1[1], i0[2]) * wx1;
        double c01 = DV(i0[0], i0[1], i1[2]) * wx0 + DV(i1[0], i0[1], i1[2]) * wx1;
        double c11 = DV(i0[0], i1[1], i1[2]) * wx0 + DV(i1[0], i1[1], i1[2]) * wx1;
        double c0 = c00 * wy0 + c10 * wy1;
        double c1 = c01 * wy0 + c11 * wy1;
        delta[p] = c0 * wz0 + c1 * wz1;
#undef DV
    }
}

void orc_cutoffs(int64_t n, const double *delta, double rc_min, double rc_max, double ramp,
                 double *rc) {
    for (int64_t p = 0; p < n; ++p) {
        double q = delta[p] / ramp;
        if (q > 1.0) q = 1.0;
        rc[p] = rc_max - (rc_max - rc_min) * q;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 9: linked cells (Section 2.3): cells of edge >= l, n_a = floor(L_a/l)*/
/* ------------------------------------------------------------------------ */
void orc_cell_dims(const double *L, double l, int32_t *nc) {
    for (int a = 0; a < 3; ++a) {
        int32_t k = (int32_t)floor(L[a] / l);
        nc[a] = k < 1 ? 1 : k;
    }
}

void orc_cells(int64_t n, const double *x, const double *y, const double *z, const double *L,
               const int32_t *nc, int32_t *cell_of, int32_t *cell_start) {
    double sx = (double)nc[0] / L[0], sy = (double)nc[1] / L[1], sz = (double)nc[2] / L[2];
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    memset(cell_start, 0, (size_t)(ncell + 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_index_1d(wrap1(x[i], L[0]), sx, nc[0]);
        int64_t cy = cell_index_1d(wrap1(y[i], L[1]), sy, nc[1]);
        int64_t cz = cell_index_1d(wrap1(z[i], L[2]), sz, nc[2]);
        int32_t c = (int32_t)((cz * nc[1] + cy) * nc[0] + cx);
        cell_of[i] = c;
        cell_start[c + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
}

/* ------------------------------------------------------------------------ */
/* Step 10: the truncated Lennard-Jones 12-6 pair sum with per-particle      */
/* cutoffs (Eqs. 2-3, Algorithm 2.3), over ALL j for each listed i (O(N^2)), */
/* minimum image d -= L*rint(d/L).                                           */
/*   rule 0 (Algorithm 2.3): j acts on i iff r^2 < rc_i^2, no Newton-3 term;  */
/*   rule 1: iff r^2 <= max(rc_i, rc_j)^2 (symmetric).                        */
/* For an included pair, with s2 = sigma^2/r^2 and s6 = s2^3:                */
/*   U = 4 eps s6 (s6 - 1), F_i += 24 eps s6 (2 s6 - 1)/r^2 * d  (d = x_i-x_j)*/
/*   E += U/2,  W_ab += d_a d_b f/2  (each ordered pair counts one half).     */
/* idx lists the i to evaluate (NULL: all n); outputs are per listed i;      */
/* E and W are summed over the listed i only.                                */
/* ------------------------------------------------------------------------ */
void orc_forces(int64_t n, const double *x, const double *y, const double *z, const double *rc,
                const double *L, double eps, double sigma, int rule,
                const int64_t *idx, int64_t nidx,
                double *fx, double *fy, double *fz, int32_t *nnbr,
                double *e_out, double *w_out) {
    if (!idx) nidx = n;
    double *ei = (double *)calloc((size_t)(nidx > 0 ? nidx : 1), sizeof(double));
    double *wi = (double *)calloc((size_t)(nidx > 0 ? nidx : 1) * 6, sizeof(double));
    double sig2 = sigma * sigma;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nidx; ++q) {
        int64_t i = idx ? idx[q] : q;
        ksum Fx = {0, 0}, Fy = {0, 0}, Fz = {0, 0}, E = {0, 0};
        ksum W[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        int32_t cnt = 0;
        double xi = x[i], yi = y[i], zi = z[i], rci = rc[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
            dx = dx - L[0] * rint(dx / L[0]);
            dy = dy - L[1] * rint(dy / L[1]);
            dz = dz - L[2] * rint(dz / L[2]);
            double r2 = (dx * dx + dy * dy) + dz * dz;
            int inc;
            if (rule == 0) {
                inc = r2 < rci * rci;
            } else {
                double m = rci > rc[j] ? rci : rc[j];
                inc = r2 <= m * m;
            }
            if (!inc) continue;
            double r2i = 1.0 / r2;
            double s2 = sig2 * r2i;
            double s6 = s2 * s2 * s2;
            double fpair = 24.0 * eps * s6 * (2.0 * s6 - 1.0) * r2i;
            double u = 4.0 * eps * s6 * (s6 - 1.0);
            ks_add(&Fx, fpair * dx);
            ks_add(&Fy, fpair * dy);
            ks_add(&Fz, fpair * dz);
            ks_add(&E, 0.5 * u);
            ks_add(&W[0], 0.5 * dx * dx * fpair);
            ks_add(&W[1], 0.5 * dy * dy * fpair);
            ks_add(&W[2], 0.5 * dz * dz * fpair);
            ks_add(&W[3], 0.5 * dx * dy * fpair);
            ks_add(&W[4], 0.5 * dx * dz * fpair);
            ks_add(&W[5], 0.5 * dy * dz * fpair);
            ++cnt;
        }
        fx[q] = ks_val(&Fx);
        fy[q] = ks_val(&Fy);
        fz[q] = ks_val(&Fz);
        if (nnbr) nnbr[q] = cnt;
        ei[q] = ks_val(&E);
        for (int c = 0; c < 6; ++c) wi[q * 6 + c] = ks_val(&W[c]);
    }
    ksum Et = {0, 0};
    ksum Wt[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int64_t q = 0; q < nidx; ++q) {
        ks_add(&Et, ei[q]);
        for (int c = 0; c < 6; ++c) ks_add(&Wt[c], wi[q * 6 + c]);
    }
    if (e_out) *e_out = ks_val(&Et);
    if (w_out) for (int c = 0; c < 6; ++c) w_out[c] = ks_val(&Wt[c]);
    free(ei);
    free(wi);
}

/* ------------------------------------------------------------------------ */
/* Step 11: velocity Verlet (Fig. 3, box 5), FP64, mass m.                   */
/*   kick:  v += (0.5 dt / m) F        drift: x += dt v, then wrap           */
/* ------------------------------------------------------------------------ */
void orc_kick(int64_t n, double *vx, double *vy, double *vz, const double *fx,
              const double *fy, const double *fz, double dt, double mass) {
    double c = (0.5 * dt) / mass;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] = vx[i] + c * fx[i];
        vy[i] = vy[i] + c * fy[i];
        vz[i] = vz[i] + c * fz[i];
    }
}

void orc_drift(int64_t n, double *x, double *y, double *z, const double *vx, const double *vy,
               const double *vz, double dt, const double *L) {
    for (int64_t i = 0; i < n; ++i) {
        x[i] = wrap1(x[i] + dt * vx[i], L[0]);
        y[i] = wrap1(y[i] + dt * vy[i], L[1]);
        z[i] = wrap1(z[i] + dt * vz[i], L[2]);
    }
}
