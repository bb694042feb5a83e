/*
 * CPU oracle for the scatter-limited hybrid (Q)MC / DG-S_N transport method
 * (Krotz & McClarren, "Scatter-Limited Hybrid Monte Carlo, Deterministic
 * Transport with Quasi-Monte Carlo Sampling", arXiv:2511.16821).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, sequential
 * reference that the device library is checked against.  Nothing in the
 * product path links, loads or calls it; only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark do.  It shares no code, header, table
 * or constant generator with the device library.
 *
 * Everything is FP64, single threaded, in particle-index order, compiled with
 * -ffp-contract=off.  Each function names the passage of the paper it follows.
 *
 * Readings of the paper that this file fixes (the paper is silent, garbled or
 * inconsistent there) are listed in the design notes; in short:
 *   - phi = integral of Psi over the sphere; Q is the angle-integrated source,
 *     so the angular source is Q/(4 pi) (Sec. 2.1, eq. (1) with Sec. 2.3).
 *   - 2-D means x-y geometry invariant in z with directions on the full sphere;
 *     path length is the 3-D length c*t, in-plane motion is (Ox, Oy)*s.
 *   - the track-length estimator is the exact integral of the exponentially
 *     decaying implicit-capture weight, w (1 - exp(-sigma l)) / sigma, so that
 *     sigma * contribution equals the weight lost on the segment.
 *   - one optical depth tau = -ln u per flight, consumed at rate sigma_s across
 *     cells (Sec. 2.3, "sample next scatter at rate sigma_s").
 *   - the remap (step 3 of Sec. 2.2) emits from Q + sigma_s (phi_pre + phi_post
 *     + phi_c), with phi_c bilinear per cell from the DG solve.  Emission (both
 *     passes) is stratified by cell: with M_i = A dt qbar_i (qbar_i the
 *     largest corner |q_i| rounded up to a power of two) and w_q = sum(M)/N_p
 *     (the correctly rounded sum) rounded down to five significant bits, cell
 *     i receives floor(r_i) or floor(r_i) + 1 particles, r_i = M_i / w_q,
 *     the second with probability frac(r_i) (a point of the cell's own count
 *     stream decides); each particle is uniform in its cell with weight
 *     w_q q(x,y) / qbar_i, and draws its points from its cell's own stream at
 *     its index within the cell, so a change of one cell's count moves no
 *     other particle.
 *
 * Parity unpinned (no closed form or independent check exists): none of the
 * functions below; the tests pin each one (points, attenuation, Erlang split,
 * balance, DG manufactured solution, remap weights, thinning).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Point generator (Sec. 2.4: low-discrepancy points replace pseudo-random     */
/* draws inside the same inverse-CDF maps).  Sobol' digital sequence in        */
/* natural (not Gray-code) index order, nested (Owen-type) scrambled with the  */
/* hash permutation of Laine & Karras (2011) on bit-reversed digits, as        */
/* described by Burley (2020).  Stream seeds and pseudo-random mode use the    */
/* SplitMix64 output function (Steele, Lea & Flood 2014).                      */
/* ------------------------------------------------------------------------ */

uint64_t or_mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Stream of points for (time step, pass, population, cohort). */
uint64_t or_stream_seed(uint64_t seed, uint64_t step, uint32_t pass,
                        uint32_t pop, uint64_t cohort)
{
    uint64_t h = or_mix64(seed);
    h = or_mix64(h ^ step);
    h = or_mix64(h ^ (uint64_t)(pass * 16u + pop));
    h = or_mix64(h ^ cohort);
    return h;
}

static uint32_t or_reverse_bits(uint32_t x)
{
    uint32_t r = 0;
    for (int b = 0; b < 32; ++b)
        if (x & (1u << b)) r |= 1u << (31 - b);
    return r;
}

/* Nested scramble: output digit k (from the most significant) depends only on
 * input digits 1..k.  On the bit-reversed word, adding a seed and x ^= x * even
 * only propagate information from low bits to high bits. */
uint32_t or_nested_scramble(uint32_t x, uint32_t s)
{
    x = or_reverse_bits(x);
    x += s;
    x ^= x * 0x6c50b47cu;
    x ^= x * 0xb82f1e52u;
    x ^= x * 0xc7afe638u;
    x ^= x * 0x8d22f6e6u;
    return or_reverse_bits(x);
}

/* Unscrambled Sobol' word: XOR of the direction numbers selected by the bits
 * of the index (natural order).  V holds 32 words per dimension. */
uint32_t or_sobol_word(const uint32_t *V, uint32_t dim, uint32_t index)
{
    uint32_t x = 0;
    for (int j = 0; j < 32; ++j)
        if ((index >> j) & 1u) x ^= V[dim * 32u + (uint32_t)j];
    return x;
}

/* Halton sequence (Halton 1960; the point set the paper uses, Sec. 2.4):
 * coordinate d of point i is the radical inverse of i in the d-th prime base
 * b, phi_b(i) = sum_k a_k b^-(k+1) for i = sum_k a_k b^k.  Returned as the
 * 32-bit word floor(phi_b(i) 2^32): with R the digit-reversed integer and
 * D = b^K (K digits), phi_b(i) = R / D, and the floor is taken in two exact
 * integer divisions (R < D < 2^40). */
enum { OR_HALTON_DIMS = 32 };
static const uint32_t or_primes[OR_HALTON_DIMS] = {
    2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53,
    59, 61, 67, 71, 73, 79, 83, 89, 97, 101, 103, 107, 109, 113, 127, 131};

uint32_t or_halton_u32(uint32_t dim, uint32_t index)
{
    const uint64_t b = or_primes[dim];
    uint64_t R = 0, D = 1;
    for (uint32_t i = index; i > 0; i /= (uint32_t)b) {
        R = R * b + (uint64_t)(i % (uint32_t)b);
        D *= b;
    }
    const uint64_t q1 = (R << 24) / D, r1 = (R << 24) % D;
    return (uint32_t)((q1 << 8) + ((r1 << 8) / D));
}

typedef struct {
    int mode;             /* 0 = scrambled Sobol', 1 = pseudo-random,  */
                          /* 2 = randomly shifted Halton               */
    int sobol_dims;       /* dimensions available in V                 */
    const uint32_t *V;    /* direction numbers, [sobol_dims][32]       */
} or_points;

uint32_t or_point_u32(const or_points *P, uint64_t stream, uint32_t dim,
                      uint32_t index)
{
    if (P->mode == 0 && (int)dim < P->sobol_dims) {
        uint32_t s = (uint32_t)(or_mix64(stream + dim) >> 32);
        return or_nested_scramble(or_sobol_word(P->V, dim, index), s);
    }
    if (P->mode == 2 && dim < OR_HALTON_DIMS) {
        /* randomised by a shift modulo 1 (Cranley & Patterson 1976) per
         * (stream, dimension) */
        uint32_t s = (uint32_t)(or_mix64(stream + dim) >> 32);
        return or_halton_u32(dim, index) + s;
    }
    uint64_t ctr = ((uint64_t)dim << 32) | (uint64_t)index;
    return (uint32_t)(or_mix64(stream ^ or_mix64(ctr)) >> 32);
}

/* u in (0,1): never 0, never 1. */
double or_u01(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

/* ------------------------------------------------------------------------ */
/* Scatter-limited Monte Carlo pass (Sec. 2.3).                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny;
    double x_lo, x_hi, y_lo, y_hi;
    const double *sig_s, *sig_a; /* per cell, row-major j*nx+i */
    double c, dt;
    const int32_t *ns_cell;      /* per-cell scatter limits (-1 unlimited), or NULL */
    int bc;                      /* reflective sides: bit 0 x_lo, 1 x_hi, 2 y_lo, 3 y_hi */
    int steady;                  /* 1: steady state (one infinite time step, Sec. 3) */
    double horizon;              /* steady state: path length at which a history ends */
    int census_qmc;              /* census histories: 1 cell cohorts, 0 a stream each */
    /* prescribed isotropic inflow G on the boundary faces (Sec. 2.1), or
     * NULL: 2 ny + 2 nx values, the x_lo faces (j = 0..ny-1), the x_hi
     * faces, the y_lo faces (i = 0..nx-1), the y_hi faces */
    const double *inflow;
} or_mesh;

/* Boundary faces as emitters: face f of the inflow array, its side (0 x_lo,
 * 1 x_hi, 2 y_lo, 3 y_hi) and its index along the side. */
static int or_face_side(int f, int nx, int ny, int *k)
{
    if (f < ny) { *k = f; return 0; }
    if (f < 2 * ny) { *k = f - ny; return 1; }
    if (f < 2 * ny + nx) { *k = f - 2 * ny; return 2; }
    *k = f - 2 * ny - nx;
    return 3;
}

double or_pow2_ceil(double v);

/* Majorants of the boundary faces: the particles entering through face f
 * in a step carry the partial current of an isotropic inflow, the integral
 * over the inward half-sphere of (Omega . n) G = pi G per unit length and
 * time, so M_f = (pi L_f) tdt pow2_ceil(|G_f|), with L_f the face length
 * and tdt the step (1 in steady state, per unit time). */
void or_face_majorants(const double *inflow, int nx, int ny, double hx, double hy, double tdt,
                       double *M)
{
    const double cx = (M_PI * hy) * tdt, cy = (M_PI * hx) * tdt;
    for (int f = 0; f < 2 * (nx + ny); ++f) {
        int k;
        const int side = or_face_side(f, nx, ny, &k);
        M[f] = (side < 2 ? cx : cy) * or_pow2_ceil(fabs(inflow[f]));
    }
}

enum { OR_BC_XLO = 1, OR_BC_XHI = 2, OR_BC_YLO = 4, OR_BC_YHI = 8 };

/* Balance record of one pass (implicit capture, Sec. 2.3). */
enum { OB_EMITTED = 0, OB_ABSORBED, OB_SCATTERED, OB_LEAKED, OB_CENSUS,
       OB_CUTOFF, OB_SOURCE_W, OB_CENSUS_IN_W, OB_N };

typedef struct {
    /* census-in bank (starts at the beginning of the step, n = 0) */
    int64_t n_in;
    const double *x, *y, *ox, *oy, *w;
    const int32_t *cell;
    const uint64_t *hid;
} or_bank_in;

typedef struct {
    /* census-out candidates at slot g (pass 2 only), size n_in + n_emit */
    double *x, *y, *ox, *oy, *w;
    int32_t *cell;
    uint64_t *hid;
    uint8_t *alive;
} or_bank_out;

/* Fraction of the segment integral: g(z) = (1 - exp(-z)) / z, g(0) = 1. */
static double or_g(double z) { return z > 0.0 ? -expm1(-z) / z : 1.0; }

/* Bilinear value of nodal data q[4] (nodes (0,0),(1,0),(0,1),(1,1)) at local
 * coordinates (a, b) in [0,1]^2, written so that equal corners give q[0]. */
static double or_bilinear(const double *q, double a, double b)
{
    return q[0] + a * (q[1] - q[0]) + b * (q[2] - q[0])
         + a * b * (q[0] - q[1] - q[2] + q[3]);
}

static double or_maxabs4(const double *q)
{
    double m = fabs(q[0]);
    for (int k = 1; k < 4; ++k) if (fabs(q[k]) > m) m = fabs(q[k]);
    return m;
}

/* Smallest power of two >= v (v > 0), 0 for v = 0.  Any majorant >= max|q|
 * keeps the emission weights unbiased; rounding it up to a power of two makes
 * it insensitive to rounding-level changes of q. */
double or_pow2_ceil(double v)
{
    if (!(v > 0.0)) return 0.0;
    int e;
    const double m = frexp(v, &e);        /* v = m 2^e, m in [0.5, 1) */
    return (m == 0.5) ? v : ldexp(1.0, e);
}

/* Majorant of cell i for the emission: M_i = adt * qbar_i, with qbar_i the
 * largest corner |q| of the cell rounded up to a power of two (a majorant of
 * |q| over the cell, since the bilinear q takes its extremes at the corners). */
void or_cell_majorants(const double *q_nodal, int64_t n, double adt, double *M)
{
    for (int64_t i = 0; i < n; ++i) M[i] = adt * or_pow2_ceil(or_maxabs4(q_nodal + 4 * i));
}

/* v rounded down to five significant bits (v > 0): with m in [1/2, 1) and
 * v = m 2^e, floor(32 m) / 32 * 2^e.  Every step is exact. */
double or_quantum(double v)
{
    if (!(v > 0.0)) return 0.0;
    int e;
    const double m = frexp(v, &e);
    return ldexp(floor(m * 32.0) / 32.0, e);
}

/* Emission counts of one pass (Sec. 2.3: particles are born in proportion to
 * the source).  The weight quantum is w_q = quantum(total / n_src), where
 * total is the sum of the majorants M_i (the caller passes it correctly
 * rounded).  Cell i expects r_i = M_i / w_q particles and receives
 * floor(r_i) + [u_i < r_i - floor(r_i)], u_i being point 0 of dimension 0
 * of the cell's count stream (population 3 of the step's pass), so that
 * E[n_i] = r_i and the total stays close to n_src whatever the number of
 * cells.  Writes counts[i] and *wq_out; returns the total. */
int64_t or_emission_counts(const double *M, int64_t n, double total, int64_t n_src,
                           const or_points *P, uint64_t seed, uint64_t step, int kind,
                           int64_t *counts, double *wq_out)
{
    const double wq = (total > 0.0 && n_src > 0) ? or_quantum(total / (double)n_src) : 0.0;
    int64_t sum = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        if (wq > 0.0 && M[i] > 0.0) {
            const double r = M[i] / wq;
            const double fl = floor(r);
            const uint64_t cs = or_stream_seed(seed, step, (uint32_t)kind, 3u, (uint64_t)i);
            const double u = or_u01(or_point_u32(P, cs, 0, 0));
            c = (int64_t)fl + ((u < r - fl) ? 1 : 0);
        }
        counts[i] = c;
        sum += c;
    }
    if (wq_out) *wq_out = wq;
    return sum;
}

/* Identity of source particle l of cell j born in time step `step` (a
 * bijective mix of the packed (j, l) keyed by the step). */
uint64_t or_history_id(uint64_t step, int64_t j, uint32_t l)
{
    return or_mix64((((uint64_t)j << 32) | (uint64_t)l) ^ or_mix64(step));
}

enum { EV_CENSUS = 0, EV_COLLIDE = 1, EV_XFACE = 2, EV_YFACE = 3 };

/*
 * One MC pass over [t_n, t_n + dt].
 *   kind  = 1: step 1 of Sec. 2.2, the scatter-limited leg with n_lim = N_s
 *              (pre tally for n < N_s, post tally for n = N_s; n_lim < 0 means
 *              unlimited scattering, Sec. 2.3 "unlimited case").  With per-cell
 *              limits (M->ns_cell, the space-dependent N_s(x) the paper names
 *              as its next step) a segment is in the pre regime when the
 *              history's collision count is below its cell's limit; the
 *              optical depth to the next collision is kept whenever the count
 *              is below the largest limit, and is consumed only in the pre
 *              regime.
 *   kind  = 2: step 3 of Sec. 2.2, the scatter-free remap (every particle is
 *              in the post-limit regime: attenuation by sigma_t, no scatter).
 * Source: nodal (bilinear) emission density q_nodal[n_cells*4] per unit
 * area and time, angle-integrated (birth ~ q, Sec. 2.3), with counts[i]
 * particles in cell i and weight quantum wq (or_emission_counts).
 * T_a receives the pre tally, T_b the post (kind 1) or the remap tally
 * (kind 2); both are raw track-length sums (weight x length).
 * Returns the number of segments (loop iterations).
 */
int64_t or_mc_pass(const or_mesh *M, const or_points *P, int kind, int n_s,
                   const double *q_nodal, const int64_t *counts, double wq,
                   const or_bank_in *bin, uint64_t seed, uint64_t step,
                   double w_cut_rel,
                   double *T_a, double *T_b, double *bal, or_bank_out *bout)
{
    const int nx = M->nx, ny = M->ny;
    const int64_t ncell = (int64_t)nx * ny;
    const double hx = (M->x_hi - M->x_lo) / nx;
    const double hy = (M->y_hi - M->y_lo) / ny;
    /* Steady state, the infinite time step of the paper's runs (Sec. 3):
     * weights are per unit time (A in place of A dt), every particle starts
     * at path length 0, and the end of the step becomes a path horizon: the
     * time-dependent formulas below with c = 1 and dt = horizon. */
    const double c = M->steady ? 1.0 : M->c;
    const double dt = M->steady ? M->horizon : M->dt;
    const double dt_birth = M->steady ? 0.0 : M->dt;
    /* n_lim: the largest limit (draws of the optical depth); lim(cell): the
     * limit that decides the regime of a segment */
    int n_lim = (kind == 2) ? 0 : (n_s < 0 ? 0x7fffffff : n_s);
    const int32_t *nsc = (kind == 1) ? M->ns_cell : NULL;
    if (nsc) {
        n_lim = 0;
        for (int64_t i = 0; i < ncell; ++i) {
            const int v = nsc[i] < 0 ? 0x7fffffff : nsc[i];
            if (v > n_lim) n_lim = v;
        }
    }

    for (int64_t i = 0; i < ncell; ++i) { T_a[i] = 0.0; T_b[i] = 0.0; }
    for (int k = 0; k < OB_N; ++k) bal[k] = 0.0;

    /* emitters: the cells, then (with an inflow) the boundary faces */
    const int64_t n_emitters = ncell + (M->inflow ? 2 * (int64_t)(nx + ny) : 0);
    int64_t n_emit = 0;
    for (int64_t i = 0; i < n_emitters; ++i) n_emit += counts[i];
    const double w_cut = w_cut_rel * wq;

    int64_t segments = 0;
    const int64_t n_tot = bin->n_in + n_emit;
    int64_t cj = 0, cbase = 0;  /* cell of the current source particle, its first index */
    /* census cohorts: the census particles of one cell, in bank order */
    int64_t *cohort_seen = (int64_t *)calloc((size_t)(ncell > 0 ? ncell : 1), sizeof(int64_t));

    for (int64_t g = 0; g < n_tot; ++g) {
        double x, y, ox, oy, w, trel, tau = 0.0;
        int ix, iy, n = 0;
        uint64_t stream;
        uint32_t pidx, dcur;
        uint64_t hid;

        if (g < bin->n_in) {
            /* census-in particle: at t_n, scatter counter reset (Sec. 2.2, step 1) */
            x = bin->x[g]; y = bin->y[g]; ox = bin->ox[g]; oy = bin->oy[g];
            w = bin->w[g];
            ix = bin->cell[g] % nx; iy = bin->cell[g] / nx;
            hid = bin->hid[g];
            trel = 0.0;
            if (M->census_qmc) {
                /* the census cohort of its cell: the cell's census stream, at
                 * the particle's rank among the census particles of that cell
                 * in bank order (so a cohort draws one low-discrepancy point
                 * set, as the source particles of a cell do) */
                stream = or_stream_seed(seed, step, (uint32_t)kind, 1u, (uint64_t)bin->cell[g]);
                pidx = (uint32_t)cohort_seen[bin->cell[g]]++;
            } else {
                /* its own stream, keyed by its identity, point index 0 */
                stream = or_stream_seed(seed, step, (uint32_t)kind, 1u, hid);
                pidx = 0;
            }
            dcur = 0;
            bal[OB_CENSUS_IN_W] += w;
        } else {
            /* source particle l of cell j (particles in cell order): uniform
             * position in the cell and time in the step, isotropic direction,
             * signed weight w_q q(x,y) / qbar_j (qbar_j the cell's power-of-two
             * majorant of |q|, so |w| <= w_q and, with E[n_j] = M_j / w_q,
             * the expected weight of the cell is its integral of q over the
             * step); points of the cell's stream at index l. */
            const int64_t s = g - bin->n_in;
            while (s >= cbase + counts[cj]) { cbase += counts[cj]; cj += 1; }
            const int64_t ci = cj;
            const uint32_t l = (uint32_t)(s - cbase);
            stream = or_stream_seed(seed, step, (uint32_t)kind, 0u, (uint64_t)ci);
            pidx = l;
            hid = or_history_id(step, ci, l);
            const double u1 = or_u01(or_point_u32(P, stream, 0, pidx));
            const double u2 = or_u01(or_point_u32(P, stream, 1, pidx));
            const double u3 = or_u01(or_point_u32(P, stream, 2, pidx));
            const double u4 = or_u01(or_point_u32(P, stream, 3, pidx));
            const double u5 = or_u01(or_point_u32(P, stream, 4, pidx));
            if (ci < ncell) {
                ix = (int)(ci % nx); iy = (int)(ci / nx);
                x = M->x_lo + hx * ((double)ix + u1);
                y = M->y_lo + hy * ((double)iy + u2);
                trel = u3 * dt_birth;
                const double st = 2.0 * sqrt(u4 * (1.0 - u4)); /* sin(theta), Oz = 1 - 2 u4 */
                const double ph = 2.0 * M_PI * u5;
                ox = st * cos(ph);
                oy = st * sin(ph);
                const double *qc = q_nodal + 4 * ci;
                w = or_bilinear(qc, u1, u2) * (wq / or_pow2_ceil(or_maxabs4(qc)));
            } else {
                /* entering through boundary face f (Sec. 2.1 inflow G):
                 * uniform along the face (dim 0) and in time (dim 1), the
                 * cosine law about the inward normal, mu = sqrt(u) (dim 2),
                 * and the in-plane tangential component sqrt(1 - mu^2)
                 * cos(2 pi u) (dim 3); weight w_q G_f / pow2_ceil(|G_f|) */
                int k;
                const int f = (int)(ci - ncell);
                const int side = or_face_side(f, nx, ny, &k);
                const double mu = sqrt(u3);
                const double tg = sqrt(1.0 - u3) * cos(2.0 * M_PI * u4);
                if (side < 2) {
                    ix = side == 0 ? 0 : nx - 1; iy = k;
                    x = M->x_lo + hx * (double)(side == 0 ? 0 : nx);
                    y = M->y_lo + hy * ((double)iy + u1);
                    ox = side == 0 ? mu : -mu;
                    oy = tg;
                } else {
                    ix = k; iy = side == 2 ? 0 : ny - 1;
                    x = M->x_lo + hx * ((double)ix + u1);
                    y = M->y_lo + hy * (double)(side == 2 ? 0 : ny);
                    oy = side == 2 ? mu : -mu;
                    ox = tg;
                }
                trel = u2 * dt_birth;
                const double G = M->inflow[f];
                w = G * (wq / or_pow2_ceil(fabs(G)));
                (void)u5;
            }
            dcur = 5;
            bal[OB_SOURCE_W] += w;
        }
        bal[OB_EMITTED] += w;
        if (n < n_lim) {
            tau = -log(or_u01(or_point_u32(P, stream, dcur, pidx)));
            dcur += 1;
        }

        for (;;) {
            const int64_t cell = (int64_t)iy * nx + ix;
            const double ss = M->sig_s[cell], sa = M->sig_a[cell], st = sa + ss;
            const int lim = nsc ? (nsc[cell] < 0 ? 0x7fffffff : nsc[cell]) : n_lim;
            const int pre = (n < lim);
            double d_cen = c * (dt - trel);
            if (d_cen < 0.0) d_cen = 0.0;
            double d_col = INFINITY;
            if (pre && ss > 0.0) { d_col = tau / ss; if (d_col < 0.0) d_col = 0.0; }
            double d_x = INFINITY, d_y = INFINITY;
            if (ox > 0.0) d_x = (M->x_lo + hx * (double)(ix + 1) - x) / ox;
            else if (ox < 0.0) d_x = (M->x_lo + hx * (double)ix - x) / ox;
            if (oy > 0.0) d_y = (M->y_lo + hy * (double)(iy + 1) - y) / oy;
            else if (oy < 0.0) d_y = (M->y_lo + hy * (double)iy - y) / oy;
            if (d_x < 0.0) d_x = 0.0;
            if (d_y < 0.0) d_y = 0.0;

            /* nearest event; ties: census > collision > x face > y face */
            double l = d_cen; int ev = EV_CENSUS;
            if (d_col < l) { l = d_col; ev = EV_COLLIDE; }
            if (d_x < l) { l = d_x; ev = EV_XFACE; }
            if (d_y < l) { l = d_y; ev = EV_YFACE; }

            /* implicit capture with sigma_a before the limit, sigma_t after */
            const double sig = pre ? sa : st;
            const double z = sig * l;
            const double contrib = w * l * or_g(z);
            if (pre) T_a[cell] += contrib; else T_b[cell] += contrib;
            bal[OB_ABSORBED] += sa * contrib;
            if (!pre) bal[OB_SCATTERED] += ss * contrib;
            w = w * exp(-z);
            if (pre && ss > 0.0) tau -= ss * l;
            x += ox * l;
            y += oy * l;
            trel += l / c;
            segments += 1;

            if (ev == EV_CENSUS) {
                bal[OB_CENSUS] += w;
                if (bout) {
                    bout->x[g] = x; bout->y[g] = y; bout->ox[g] = ox; bout->oy[g] = oy;
                    bout->w[g] = w; bout->cell[g] = (int32_t)cell; bout->hid[g] = hid;
                    bout->alive[g] = 1;
                }
                break;
            } else if (ev == EV_COLLIDE) {
                /* isotropic re-emission, counter n <- n + 1 (Sec. 2.3) */
                const double ua = or_u01(or_point_u32(P, stream, dcur, pidx));
                const double ub = or_u01(or_point_u32(P, stream, dcur + 1, pidx));
                dcur += 2;
                const double stn = 2.0 * sqrt(ua * (1.0 - ua));
                const double ph = 2.0 * M_PI * ub;
                ox = stn * cos(ph);
                oy = stn * sin(ph);
                n += 1;
                if (n < n_lim) {
                    tau = -log(or_u01(or_point_u32(P, stream, dcur, pidx)));
                    dcur += 1;
                }
            } else if (ev == EV_XFACE) {
                /* a reflective side mirrors the direction (specular
                 * reflection): the history stays in its cell */
                if (ox > 0.0) {
                    x = M->x_lo + hx * (double)(ix + 1);
                    if (ix == nx - 1 && (M->bc & OR_BC_XHI)) ox = -ox; else ix += 1;
                } else {
                    x = M->x_lo + hx * (double)ix;
                    if (ix == 0 && (M->bc & OR_BC_XLO)) ox = -ox; else ix -= 1;
                }
                if (ix < 0 || ix >= nx) { bal[OB_LEAKED] += w; break; }
            } else {
                if (oy > 0.0) {
                    y = M->y_lo + hy * (double)(iy + 1);
                    if (iy == ny - 1 && (M->bc & OR_BC_YHI)) oy = -oy; else iy += 1;
                } else {
                    y = M->y_lo + hy * (double)iy;
                    if (iy == 0 && (M->bc & OR_BC_YLO)) oy = -oy; else iy -= 1;
                }
                if (iy < 0 || iy >= ny) { bal[OB_LEAKED] += w; break; }
            }
            if (fabs(w) < w_cut) { bal[OB_CUTOFF] += w; break; }
        }
    }
    free(cohort_seen);
    return segments;
}

/* ------------------------------------------------------------------------ */
/* Census population control.  The paper runs steady state only and does not  */
/* say how the census is capped; the reading recorded in the design notes:    */
/* when more than cap particles reach t_{n+1}, each survivor is kept with     */
/* probability p_q and its weight divided by p_q, where p_q is                */
/* (cap - margin) / count rounded DOWN to 11 significant bits and             */
/* margin = ceil(4 sqrt(cap)) + 16.  The Bernoulli draw compares the          */
/* particle's 64-bit key mix64(thin_stream ^ hid) with p_q 2^64, so a         */
/* survivor's fate depends on its own id and on p_q only; rounding p_q to a    */
/* coarse grid keeps it unchanged when the count moves by a few particles.    */
/* In the rare event that more than cap survive the draw, the first cap in    */
/* slot order are kept (and the overflow is reported).                       */
/* ------------------------------------------------------------------------ */

/* p_q = p rounded down to 11 significant bits, as mant * 2^shift with
 * 1024 <= mant < 2048; the keep test is (key >> (64 + shift)) < mant. */
void or_thin_prob(int64_t count, int64_t cap, double *p_q, int *keep_shift,
                  uint64_t *keep_mant)
{
    int64_t margin = (int64_t)ceil(4.0 * sqrt((double)cap)) + 16;
    int64_t target = cap - margin;
    if (target < 1) target = 1;
    const double p = (double)target / (double)count;
    int k;
    const double m = frexp(p, &k);             /* p = m 2^k, m in [0.5, 1) */
    const double mant = floor(ldexp(m, 11));   /* in [1024, 2048)          */
    *keep_mant = (uint64_t)mant;
    *keep_shift = k - 11;                      /* p_q = mant 2^(k - 11)    */
    *p_q = ldexp(mant, k - 11);
}

/* keep[g] = 1 for the kept candidates (slot order); returns the kept count,
 * writes the weight factor 1/p_q (1 if no thinning) and the overflow flag. */
int64_t or_thin(int64_t n_cand, const uint8_t *alive, const uint64_t *hid,
                int64_t cap, uint64_t thin_stream, uint8_t *keep, double *factor,
                int *overflow)
{
    int64_t count = 0;
    for (int64_t g = 0; g < n_cand; ++g) { keep[g] = 0; if (alive[g]) ++count; }
    *overflow = 0;
    if (count <= cap) {
        for (int64_t g = 0; g < n_cand; ++g) keep[g] = alive[g];
        *factor = 1.0;
        return count;
    }
    double p_q;
    int sh;
    uint64_t mant;
    or_thin_prob(count, cap, &p_q, &sh, &mant);
    const int rs = 64 + sh;  /* key < mant 2^(64+sh)  <=>  (key >> rs) < mant */
    int64_t kept = 0;
    for (int64_t g = 0; g < n_cand; ++g) {
        if (!alive[g]) continue;
        const uint64_t key = or_mix64(thin_stream ^ hid[g]);
        const uint64_t top = rs >= 64 ? 0 : (key >> rs);
        if (top < mant) {
            if (kept < cap) { keep[g] = 1; ++kept; }
            else *overflow = 1;
        }
    }
    *factor = 1.0 / p_q;
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Discrete-ordinates collided solve with bilinear discontinuous Galerkin     */
/* (step 2 of Sec. 2.2, eq. for the super-N_s flux; S_N estimator of <Psi>    */
/* by the quadrature of the ordinates).  Per direction (a, b) = (Ox, Oy) and   */
/* cell K, find psi in Q1(K) with, for every test function v in Q1(K),         */
/*   int_K (a psi_x + b psi_y) v + sig_e int_K psi v                          */
/*     + sum_{inflow faces} |Omega.n| int_F psi v                             */
/*   = int_K S v + sum_{inflow faces} |Omega.n| int_F psi_upwind v,           */
/* integrated exactly by the 2-point Gauss rule in each direction.            */
/* Local node k = ix + 2*iy at (x_{ix}, y_{iy}) of the cell.                  */
/* ------------------------------------------------------------------------ */

static double or_L(int i, double t) { return i ? t : 1.0 - t; }
static double or_dL(int i) { return i ? 1.0 : -1.0; }

/* Solve the 4x4 system A u = r by Gaussian elimination, partial pivoting. */
static int or_solve4(double A[4][4], double r[4], double u[4])
{
    int perm[4] = {0, 1, 2, 3};
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int row = col + 1; row < 4; ++row)
            if (fabs(A[row][col]) > fabs(A[piv][col])) piv = row;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col) {
            for (int k = 0; k < 4; ++k) { double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t; }
            double t = r[col]; r[col] = r[piv]; r[piv] = t;
            int tp = perm[col]; perm[col] = perm[piv]; perm[piv] = tp;
        }
        for (int row = col + 1; row < 4; ++row) {
            const double f = A[row][col] / A[col][col];
            for (int k = col; k < 4; ++k) A[row][k] -= f * A[col][k];
            r[row] -= f * r[col];
        }
    }
    for (int row = 3; row >= 0; --row) {
        double s = r[row];
        for (int k = row + 1; k < 4; ++k) s -= A[row][k] * u[k];
        u[row] = s / A[row][row];
    }
    (void)perm;
    return 0;
}

/*
 * One transport sweep for the single direction (a, b): solves every cell in
 * upwind order.  sig_e per cell, src nodal [n_cells*4].  Inflow data on the
 * domain boundary: in_x[j*2 + iy] on the x-inflow side (row j, node iy), and
 * in_y[i*2 + ix] on the y-inflow side; NULL means vacuum (zero inflow).
 * psi [n_cells*4] receives the nodal solution.
 */
int or_dg_sweep(int nx, int ny, double x_lo, double x_hi, double y_lo, double y_hi,
                const double *sig_e, double a, double b, const double *src,
                const double *in_x, const double *in_y, double *psi)
{
    const double hx = (x_hi - x_lo) / nx, hy = (y_hi - y_lo) / ny;
    const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const double gw = 0.5; /* weight per point on [0,1] */

    for (int jj = 0; jj < ny; ++jj) {
        const int j = (b > 0.0) ? jj : ny - 1 - jj;
        for (int ii = 0; ii < nx; ++ii) {
            const int i = (a > 0.0) ? ii : nx - 1 - ii;
            const int64_t cell = (int64_t)j * nx + i;
            double A[4][4], r[4], u[4];
            memset(A, 0, sizeof A);
            memset(r, 0, sizeof r);
            const double *S = src + 4 * cell;
            /* volume terms */
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) {
                    const double xi = gp[p], eta = gp[q];
                    const double wv = gw * gw * hx * hy;
                    double Sv = 0.0;
                    for (int k = 0; k < 4; ++k)
                        Sv += S[k] * or_L(k & 1, xi) * or_L(k >> 1, eta);
                    for (int ti = 0; ti < 4; ++ti) {
                        const double vt = or_L(ti & 1, xi) * or_L(ti >> 1, eta);
                        r[ti] += wv * Sv * vt;
                        for (int tj = 0; tj < 4; ++tj) {
                            const double N = or_L(tj & 1, xi) * or_L(tj >> 1, eta);
                            const double Nx = or_dL(tj & 1) / hx * or_L(tj >> 1, eta);
                            const double Ny = or_L(tj & 1, xi) * or_dL(tj >> 1) / hy;
                            A[ti][tj] += wv * ((a * Nx + b * Ny) * vt + sig_e[cell] * N * vt);
                        }
                    }
                }
            /* x-inflow face: xi_f = 0 if a > 0 (left), 1 if a < 0 (right) */
            {
                const int fx = (a > 0.0) ? 0 : 1;
                const double xi = (double)fx;
                for (int q = 0; q < 2; ++q) {
                    const double eta = gp[q];
                    const double wf = gw * hy * fabs(a);
                    double up = 0.0;
                    const int inb = (a > 0.0) ? i - 1 : i + 1;
                    if (inb >= 0 && inb < nx) {
                        /* neighbour's face on our side is its xi = 1 - fx */
                        const double *pn = psi + 4 * ((int64_t)j * nx + inb);
                        const int nf = 1 - fx;
                        up = pn[nf + 0] * or_L(0, eta) + pn[nf + 2] * or_L(1, eta);
                    } else if (in_x) {
                        up = in_x[2 * j + 0] * or_L(0, eta) + in_x[2 * j + 1] * or_L(1, eta);
                    }
                    for (int ti = 0; ti < 4; ++ti) {
                        const double vt = or_L(ti & 1, xi) * or_L(ti >> 1, eta);
                        r[ti] += wf * up * vt;
                        for (int tj = 0; tj < 4; ++tj)
                            A[ti][tj] += wf * or_L(tj & 1, xi) * or_L(tj >> 1, eta) * vt;
                    }
                }
            }
            /* y-inflow face: eta_f = 0 if b > 0 (bottom), 1 if b < 0 (top) */
            {
                const int fy = (b > 0.0) ? 0 : 1;
                const double eta = (double)fy;
                for (int p = 0; p < 2; ++p) {
                    const double xi = gp[p];
                    const double wf = gw * hx * fabs(b);
                    double up = 0.0;
                    const int jnb = (b > 0.0) ? j - 1 : j + 1;
                    if (jnb >= 0 && jnb < ny) {
                        const double *pn = psi + 4 * ((int64_t)jnb * nx + i);
                        const int nf = 1 - fy;
                        up = pn[2 * nf + 0] * or_L(0, xi) + pn[2 * nf + 1] * or_L(1, xi);
                    } else if (in_y) {
                        up = in_y[2 * i + 0] * or_L(0, xi) + in_y[2 * i + 1] * or_L(1, xi);
                    }
                    for (int ti = 0; ti < 4; ++ti) {
                        const double vt = or_L(ti & 1, xi) * or_L(ti >> 1, eta);
                        r[ti] += wf * up * vt;
                        for (int tj = 0; tj < 4; ++tj)
                            A[ti][tj] += wf * or_L(tj & 1, xi) * or_L(tj >> 1, eta) * vt;
                    }
                }
            }
            if (or_solve4(A, r, u) != 0) return -1;
            for (int k = 0; k < 4; ++k) psi[4 * cell + k] = u[k];
        }
    }
    return 0;
}

/*
 * One source iteration of the collided solve (step 2 of Sec. 2.2): with the
 * nodal iterate phi [n_cells*4], sweep every direction with the source
 * sig_s/(4 pi) (phi + phi_post) and return acc = sum_m w_m psi_m.  The
 * reflected traces lag one iteration: out_x/out_y hold each direction's
 * outflow traces on its downwind x and y sides (two nodes per row or column)
 * from the previous call (zero before the first) and are replaced by this
 * iteration's.  sig_e per cell as in or_dg_collided.  Returns 0, or -1 when a
 * cell system is singular.
 */
int or_dg_one_iteration(const or_mesh *M, const double *sig_e, int n_dir,
                        const double *dox, const double *doy, const double *dw,
                        const int *refl_x, const int *refl_y, const double *phi_post,
                        const double *phi, double *out_x, double *out_y, double *acc)
{
    const int nx = M->nx, ny = M->ny;
    const int64_t ncell = (int64_t)nx * ny;
    const size_t nn = (size_t)ncell * 4;
    const size_t bx = (size_t)2 * ny, by = (size_t)2 * nx;
    double *src = (double *)malloc(sizeof(double) * nn);
    double *psi = (double *)malloc(sizeof(double) * nn);
    double *prev_x = (double *)malloc(sizeof(double) * (size_t)n_dir * bx);
    double *prev_y = (double *)malloc(sizeof(double) * (size_t)n_dir * by);
    int rc = 0;
    for (int64_t i = 0; i < ncell; ++i)
        for (int k = 0; k < 4; ++k)
            src[4 * i + k] = M->sig_s[i] / (4.0 * M_PI) * (phi[4 * i + k] + phi_post[i]);
    for (size_t k = 0; k < nn; ++k) acc[k] = 0.0;
    memcpy(prev_x, out_x, sizeof(double) * (size_t)n_dir * bx);
    memcpy(prev_y, out_y, sizeof(double) * (size_t)n_dir * by);
    for (int m = 0; m < n_dir; ++m) {
        const int rx = (dox[m] > 0.0) ? (M->bc & OR_BC_XLO) : (M->bc & OR_BC_XHI);
        const int ry = (doy[m] > 0.0) ? (M->bc & OR_BC_YLO) : (M->bc & OR_BC_YHI);
        const double *in_x = rx ? prev_x + (size_t)refl_x[m] * bx : NULL;
        const double *in_y = ry ? prev_y + (size_t)refl_y[m] * by : NULL;
        if (or_dg_sweep(nx, ny, M->x_lo, M->x_hi, M->y_lo, M->y_hi, sig_e,
                        dox[m], doy[m], src, in_x, in_y, psi) != 0) {
            rc = -1;
            break;
        }
        for (size_t k = 0; k < nn; ++k) acc[k] += dw[m] * psi[k];
        /* outflow traces: x side xi = 1 (nodes 1, 3) if Ox > 0 else xi = 0
         * (nodes 0, 2); y side eta = 1 (nodes 2, 3) if Oy > 0 else 0 (0, 1) */
        const int ib = (dox[m] > 0.0) ? nx - 1 : 0, fx = (dox[m] > 0.0) ? 1 : 0;
        for (int j = 0; j < ny; ++j) {
            const double *pc = psi + 4 * ((int64_t)j * nx + ib);
            out_x[(size_t)m * bx + 2 * j] = pc[fx];
            out_x[(size_t)m * bx + 2 * j + 1] = pc[fx + 2];
        }
        const int jb = (doy[m] > 0.0) ? ny - 1 : 0, fy = (doy[m] > 0.0) ? 1 : 0;
        for (int i = 0; i < nx; ++i) {
            const double *pc = psi + 4 * ((int64_t)jb * nx + i);
            out_y[(size_t)m * by + 2 * i] = pc[2 * fy];
            out_y[(size_t)m * by + 2 * i + 1] = pc[2 * fy + 1];
        }
    }
    free(src); free(psi); free(prev_x); free(prev_y);
    return rc;
}

/* sigma_e = sigma_t + tau/(c dt) per cell (sigma_t in steady state). */
void or_dg_sigma_e(const or_mesh *M, double tau_closure, double *sig_e)
{
    const int64_t ncell = (int64_t)M->nx * M->ny;
    for (int64_t i = 0; i < ncell; ++i)
        sig_e[i] = M->sig_a[i] + M->sig_s[i]
                 + (M->steady ? 0.0 : tau_closure / (M->c * M->dt));
}

/*
 * Source iteration for the collided flux (step 2 of Sec. 2.2):
 *   (sig_t + tau/(c dt)) psi + Omega.grad psi = sig_s/(4 pi) (phi_c + phi_post)
 * (in steady state, M->steady, without the tau/(c dt) term)
 * with zero initial data, vacuum sides, and reflective sides (M->bc) whose
 * inflow lags one iteration (or_dg_one_iteration).  The time derivative over
 * the step is closed by tau/(c dt) (tau = 2: the step average of a flux
 * growing linearly from zero).  phi_post is cell-constant; phi_c is nodal
 * bilinear.  Stops when ||phi_new - phi_old||_2 <= tol ||phi_new||_2 (nodal
 * vectors), or, when phi_pre is given, <= tol ||phi_new + phi_pre +
 * phi_post||_2 (the whole flux of the step as the reference).
 * phi [n_cells*4] receives the result; returns the number of sweeps.
 */
int or_dg_collided(const or_mesh *M, double tau_closure, int n_dir,
                   const double *dox, const double *doy, const double *dw,
                   const int *refl_x, const int *refl_y,
                   const double *phi_post, const double *phi_pre,
                   double tol, int max_iter, double *phi, double *resid_out)
{
    const int nx = M->nx, ny = M->ny;
    const int64_t ncell = (int64_t)nx * ny;
    const size_t nn = (size_t)ncell * 4;
    double *sig_e = (double *)malloc(sizeof(double) * (size_t)ncell);
    double *acc = (double *)malloc(sizeof(double) * nn);
    const size_t bx = (size_t)2 * ny, by = (size_t)2 * nx;
    double *out_x = (double *)calloc((size_t)n_dir * bx, sizeof(double));
    double *out_y = (double *)calloc((size_t)n_dir * by, sizeof(double));
    or_dg_sigma_e(M, tau_closure, sig_e);
    for (size_t k = 0; k < nn; ++k) phi[k] = 0.0;
    int it = 0;
    double resid = 0.0;
    while (it < max_iter) {
        if (or_dg_one_iteration(M, sig_e, n_dir, dox, doy, dw, refl_x, refl_y, phi_post, phi,
                                out_x, out_y, acc) != 0) {
            it = -1;
            break;
        }
        it += 1;
        double dn = 0.0, nrm = 0.0;
        for (size_t k = 0; k < nn; ++k) {
            const double d = acc[k] - phi[k];
            const double ref = phi_pre ? acc[k] + (phi_pre[k / 4] + phi_post[k / 4]) : acc[k];
            dn += d * d;
            nrm += ref * ref;
            phi[k] = acc[k];
        }
        dn = sqrt(dn);
        nrm = sqrt(nrm);
        resid = (nrm > 0.0) ? dn / nrm : 0.0;
        if (dn <= tol * nrm) break;
    }
    if (resid_out) *resid_out = resid;
    free(sig_e); free(acc); free(out_x); free(out_y);
    return it;
}
