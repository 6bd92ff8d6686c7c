/*
 * spkmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference for the synchronous parallel
 * kinetic Monte Carlo method (spkMC) on the 3D Ising lattice (Martinez,
 * Monasterio, Marian, "Billion-atom Synchronous Parallel Kinetic Monte Carlo
 * Simulations of Critical 3D Ising Systems", arXiv:1005.4713), plus a serial
 * rejection-free BKL/n-fold simulator used as the statistical reference.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file.
 *
 * By default everything runs on one thread.  orc_set_threads(n > 1) runs the
 * per-domain loops of one cycle (the frequency lines of step 1 and the
 * decisions of steps 3-4b) as an OpenMP parallel-for; within a cycle the
 * domains read only spins no other domain writes (same-coloured octants never
 * touch), and the flips are still applied after every decision, in line
 * order, so the trajectory is bit-identical for every thread count.  It shares no code, header, table or constant generator with
 * the GPU library; the only thing both sides agree on is the published
 * definition of Philox4x32-10 and the readings of the paper listed below.
 *
 * Every step follows the paper's order and notation:
 *   - Hamiltonian H = -J sum_<ij> s_i s_j - H sum_i s_i           (Sec. 2, eq. 1)
 *   - Glauber single-spin rates (Sec. 2, eq. 3), in the detailed-balance form
 *     r = lambda / (1 + exp(beta dE)) with lambda = 1; Metropolis
 *     r = min(1, exp(-beta dE)) as a second rate family.
 *   - spkMC cycle (Sec. 3.1 steps 1-6, Sec. 3.2 steps 4a/4b):
 *       1. frequency line R_k of every subdomain            (step 1)
 *       2. R_max = max_k R_k                                (step 2)
 *       3. null event r_0k = R_max - R_k                    (step 3)
 *       4a. one sublattice (colour) for all subdomains      (step 4a)
 *       4b. event chosen with probability r/R_max           (steps 4, 4b)
 *       5. common exponential time increment                (step 5)
 *       6. boundary events become visible                   (step 6)
 *   - magnetisation (eq. 4), and the serial BKL method the paper compares to.
 *
 * Readings where the paper is silent, garbled or inconsistent (each also
 * stated where used):
 *   R1  eq. 3 is printed with tanh(2 beta dE) and dE = -J sum s_j - H s_i; only
 *       the form lambda/(1+exp(beta dE_flip)) with dE_flip the energy change of
 *       the flip satisfies detailed balance with eq. 1, so that form is used.
 *   R2  lambda = 1: time is measured in units of 1/lambda.
 *   R3  colours: each domain (edge d, even) is split into 8 octants of edge
 *       h = d/2; colour s in 0..7 names the octant (sx, sy, sz) = bits of s.
 *   R4  R_max is the maximum over the K octants of the chosen colour (the
 *       "active" reading); rmax_scope = 1 gives the all-octant reading.
 *   R5  time increment dt = -ln(xi) / (S R_max) with S the number of colours,
 *       so that every spin flips at its physical rate (step 5 is written for
 *       the case where every subdomain is active).
 *   R6  selection inside a frequency line: a single uniform u, target =
 *       u R_max, classes walked in fixed order 0..13 with running FP64 sums
 *       (separate multiply and add), the null segment last; the site is the
 *       j-th site of the chosen class in canonical order inside the octant.
 *   R7  random numbers: Philox4x32-10 counter streams (the paper only asks for
 *       independent parallel streams).
 *   R8  neighbours are counted with multiplicity (at L = 2 the +x and -x
 *       neighbour coincide and count twice).
 *   R9  two colours (Sec. 3.2, first-neighbour interactions): the cells of
 *       edge h (the octants) coloured by the parity of sx + sy + sz, a proper
 *       two-colouring of the cell lattice, so same-coloured cells never share
 *       a face; each cycle activates the 4 octants of the drawn colour in
 *       every domain, each octant its own frequency line (subdomain) with its
 *       own random stream; the colour is the top bit of the cycle word.
 *  R10  the optimistic bound R'_max of Sec. 3.2 (printed with a garbled
 *       exponent): the largest aggregate rate a region of n_k sites can have,
 *       n_k times the largest of the 14 class rates; fixed for the whole run,
 *       so no maximum over subdomains is taken.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* threads of the per-domain loops (1: plain serial loops) */
static int orc_threads = 1;
ORC_EXPORT void orc_set_threads(int32_t n) { orc_threads = n > 1 ? n : 1; }
ORC_EXPORT int32_t orc_get_threads(void) { return orc_threads; }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers: */
/* as easy as 1, 2, 3"): 10 rounds of two 32x32->64 multiplies per round,     */
/* with the key advanced by the two Weyl constants between rounds.            */
/* ------------------------------------------------------------------------- */
ORC_EXPORT void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                  uint32_t out[4]) {
    const uint32_t mult_a = 0xD2511F53u, mult_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)mult_a * (uint64_t)x0;
        uint64_t pb = (uint64_t)mult_b * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += weyl_a;
        k1 += weyl_b;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform doubles from Philox words (exact conversions, no rounding). */
ORC_EXPORT double orc_u53(uint32_t a, uint32_t b) {
    /* [0,1): 27 bits of a, 26 bits of b -> 53-bit integer / 2^53 */
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}
ORC_EXPORT double orc_uopen52(uint32_t a, uint32_t b) {
    /* (0,1): a 52-bit integer m, then (m + 1/2) / 2^52 */
    uint64_t m = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 4503599627370496.0);
}
ORC_EXPORT uint32_t orc_idx(uint32_t w, uint32_t n) {
    /* an index in [0, n) from a 32-bit word (multiply-shift) */
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

static void philox_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Parameters                                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t L;          /* lattice edge, N = L^3 sites, periodic (Sec. 4)          */
    int32_t d;          /* domain edge; octant edge h = d / 2 (reading R3)          */
    double J, H, T;     /* coupling, field, temperature (k_B = 1), eq. 1           */
    uint64_t seed;      /* Philox key                                               */
    int32_t rates;      /* 0 Glauber (eq. 3, reading R1), 1 Metropolis              */
    int32_t init;       /* 0 iid +-1 from the seed, 1 all +1, 2 all -1              */
    int32_t colours;    /* 8 = octant chessboard; 2 = octant parity (R9); 1 = the
                           whole domain is active                                   */
    int32_t rmax_scope; /* 0 = max over active lines (R4), 1 = over all octants,
                           2 = the optimistic bound R'_max (R10)                    */
    int32_t order;      /* 0 decide all then apply, 1 apply at once in domain order,
                           2 apply at once in a shuffled domain order               */
    int32_t check;      /* 1 = recompute M and B after every cycle                  */
} orc_params;

typedef struct {
    uint64_t cycle, fired, nulls;
    double t;
    int64_t M, B;
} orc_record;

/* ------------------------------------------------------------------------- */
/* Rate table (eq. 3 read as R1; Metropolis as the second family).            */
/* class c in 0..13: spin s = +1 if c >= 7 else -1; a = c mod 7 = number of   */
/* the 6 neighbours aligned with s.  Flip energy change from eq. 1:           */
/* dE = 2 J (2a - 6) + 2 H s.                                                 */
/* ------------------------------------------------------------------------- */
ORC_EXPORT int orc_rate_table(double J, double H, double T, int32_t rates, double out[14]) {
    if (!(T > 0.0) || !isfinite(T) || !isfinite(J) || !isfinite(H)) return -1;
    if (rates != 0 && rates != 1) return -1;
    double beta = 1.0 / T;
    for (int c = 0; c < 14; ++c) {
        int sgn = (c >= 7) ? 1 : -1;
        int a = c % 7;
        double dE = 2.0 * J * (double)(2 * a - 6) + 2.0 * H * (double)sgn;
        double x = beta * dE;
        double r;
        if (rates == 0) r = 1.0 / (1.0 + exp(x));
        else r = (dE <= 0.0) ? 1.0 : exp(-x);
        if (!(r > 0.0) || !isfinite(r)) return -2;
        out[c] = r;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Lattice helpers                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    int L;
    int8_t *spin; /* index x + L (y + L z) */
} lattice;

static inline int8_t sp(const lattice *g, int x, int y, int z) {
    return g->spin[(int64_t)x + (int64_t)g->L * ((int64_t)y + (int64_t)g->L * z)];
}
static inline int wrap_dec(int v, int L) { return v == 0 ? L - 1 : v - 1; }
static inline int wrap_inc(int v, int L) { return v + 1 == L ? 0 : v + 1; }

/* number of the 6 neighbours (with multiplicity) aligned with the spin */
static int aligned_count(const lattice *g, int x, int y, int z) {
    int L = g->L;
    int8_t s = sp(g, x, y, z);
    int a = 0;
    a += sp(g, wrap_dec(x, L), y, z) == s;
    a += sp(g, wrap_inc(x, L), y, z) == s;
    a += sp(g, x, wrap_dec(y, L), z) == s;
    a += sp(g, x, wrap_inc(y, L), z) == s;
    a += sp(g, x, y, wrap_dec(z, L)) == s;
    a += sp(g, x, y, wrap_inc(z, L)) == s;
    return a;
}
static int site_class(const lattice *g, int x, int y, int z) {
    return (sp(g, x, y, z) > 0 ? 7 : 0) + aligned_count(g, x, y, z);
}

/* M = sum s_i (eq. 4 times N), B = sum_i sum_{e in x,y,z} s_i s_{i+e} */
static void observables(const lattice *g, int64_t *M, int64_t *B) {
    int L = g->L;
    int64_t m = 0, b = 0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int s = sp(g, x, y, z);
                m += s;
                b += s * sp(g, wrap_inc(x, L), y, z);
                b += s * sp(g, x, wrap_inc(y, L), z);
                b += s * sp(g, x, y, wrap_inc(z, L));
            }
    *M = m;
    *B = b;
}

/* Initial state: iid spins from the Philox stream, block b = i >> 7 uses
 * counter (b_lo, b_hi, 0xFFFFFFFE, 0xFFFFFFFE); spin i is bit (i & 31) of word
 * (i >> 5) & 3, 1 -> +1, 0 -> -1. */
static void init_spins(int8_t *spin, int64_t N, uint64_t seed, int init) {
    if (init == 1 || init == 2) {
        for (int64_t i = 0; i < N; ++i) spin[i] = (int8_t)(init == 1 ? 1 : -1);
        return;
    }
    uint32_t w[4];
    int64_t last_block = -1;
    for (int64_t i = 0; i < N; ++i) {
        int64_t b = i >> 7;
        if (b != last_block) {
            philox_words(seed, (uint32_t)b, (uint32_t)((uint64_t)b >> 32), 0xFFFFFFFEu, 0xFFFFFFFEu, w);
            last_block = b;
        }
        uint32_t word = w[(i >> 5) & 3];
        spin[i] = ((word >> (i & 31)) & 1u) ? 1 : -1;
    }
}

/* ------------------------------------------------------------------------- */
/* Frequency-line selection (steps 3, 4 and 4b; reading R6).                  */
/* Running sum acc over classes 0..13 of count_c * r_c (separate multiply and */
/* add); the first class with target < acc is chosen, otherwise the null      */
/* event.  Returns 1 and the class / in-class index on a fire, 0 on a null.   */
/* ------------------------------------------------------------------------- */
static double line_total(const uint32_t hist[14], const double r[14]) {
    double acc = 0.0;
    for (int c = 0; c < 14; ++c) {
        double term = (double)hist[c] * r[c];
        acc = acc + term;
    }
    return acc;
}

ORC_EXPORT int orc_select(const uint32_t hist[14], const double r[14], double Rmax, double u,
                          uint32_t w, int32_t *cls, uint32_t *j) {
    double target = u * Rmax;
    double acc = 0.0;
    for (int c = 0; c < 14; ++c) {
        double term = (double)hist[c] * r[c];
        acc = acc + term;
        if (target < acc) {
            *cls = c;
            *j = orc_idx(w, hist[c]);
            return 1;
        }
    }
    *cls = -1;
    *j = 0;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* spkMC simulator                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    orc_params p;
    int L, d, h, nd, S;
    int64_t N;
    uint32_t K;
    double r[14];
    lattice g;
    uint32_t A;     /* active lines (octants) per domain and cycle: 1, or 4 (R9) */
    double Rbound;  /* R'_max (R10) */
    uint32_t *hist; /* K * A * 14, active lines of the current cycle */
    double *R;      /* K * A */
    uint64_t n, fired, nulls;
    double t;
    int64_t M, B;
    uint64_t check_fail;
    /* flips decided this cycle */
    int64_t *flip_site;
    int8_t *flip_old;
    int8_t *flip_a;
    uint8_t *flip_fire; /* decide-then-apply: line f fires this cycle */
    uint32_t *perm;
} orc_sim;

/* origin and edge of the active region of domain k for colour s (R3) */
static void region(const orc_sim *S, uint32_t k, int s, int *ox, int *oy, int *oz, int *edge) {
    int nd = S->nd;
    int kx = (int)(k % (uint32_t)nd), ky = (int)((k / (uint32_t)nd) % (uint32_t)nd),
        kz = (int)(k / ((uint32_t)nd * (uint32_t)nd));
    if (S->S != 1) {
        *ox = kx * S->d + (s & 1) * S->h;
        *oy = ky * S->d + ((s >> 1) & 1) * S->h;
        *oz = kz * S->d + ((s >> 2) & 1) * S->h;
        *edge = S->h;
    } else {
        *ox = kx * S->d;
        *oy = ky * S->d;
        *oz = kz * S->d;
        *edge = S->d;
    }
}

/* step 1: class histogram of one region and its frequency-line total */
static void bin_region(const orc_sim *S, uint32_t k, int s, uint32_t hist[14]) {
    int ox, oy, oz, e;
    region(S, k, s, &ox, &oy, &oz, &e);
    for (int c = 0; c < 14; ++c) hist[c] = 0;
    for (int lz = 0; lz < e; ++lz)
        for (int ly = 0; ly < e; ++ly)
            for (int lx = 0; lx < e; ++lx) hist[site_class(&S->g, ox + lx, oy + ly, oz + lz)]++;
}

/* the j-th site (0-based) of class c in canonical order q = lx + e (ly + e lz) */
static int64_t find_site(const orc_sim *S, uint32_t k, int s, int c, uint32_t j, int *a_out) {
    int ox, oy, oz, e;
    region(S, k, s, &ox, &oy, &oz, &e);
    uint32_t seen = 0;
    for (int lz = 0; lz < e; ++lz)
        for (int ly = 0; ly < e; ++ly)
            for (int lx = 0; lx < e; ++lx) {
                int x = ox + lx, y = oy + ly, z = oz + lz;
                if (site_class(&S->g, x, y, z) == c) {
                    if (seen == j) {
                        *a_out = c % 7;
                        return (int64_t)x + (int64_t)S->L * ((int64_t)y + (int64_t)S->L * z);
                    }
                    ++seen;
                }
            }
    return -1;
}

ORC_EXPORT orc_sim *orc_sim_new(const orc_params *p) {
    if (!p) return NULL;
    if (p->L < 2 || p->d < 2 || (p->d & 1) || p->L % p->d) return NULL;
    if (p->colours != 8 && p->colours != 2 && p->colours != 1) return NULL;
    if (p->colours == 1 && p->d != p->L) return NULL; /* one region only: K must be 1 */
    if (p->init < 0 || p->init > 2 || p->rmax_scope < 0 || p->rmax_scope > 2) return NULL;
    if (p->order < 0 || p->order > 2) return NULL;
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!S) return NULL;
    S->p = *p;
    S->L = p->L;
    S->d = p->d;
    S->h = p->d / 2;
    S->nd = p->L / p->d;
    S->S = p->colours;
    S->N = (int64_t)p->L * p->L * p->L;
    S->K = (uint32_t)S->nd * (uint32_t)S->nd * (uint32_t)S->nd;
    S->A = p->colours == 2 ? 4u : 1u;
    if (orc_rate_table(p->J, p->H, p->T, p->rates, S->r) != 0) {
        free(S);
        return NULL;
    }
    {   /* R10: sites of one region times the largest class rate */
        double rb = S->r[0];
        for (int c = 1; c < 14; ++c)
            if (S->r[c] > rb) rb = S->r[c];
        int e = p->colours == 1 ? S->d : S->h;
        S->Rbound = (double)((int64_t)e * e * e) * rb;
    }
    const size_t nl = (size_t)S->K * S->A;
    S->g.L = p->L;
    S->g.spin = (int8_t *)malloc((size_t)S->N);
    S->hist = (uint32_t *)calloc(nl * 14, sizeof(uint32_t));
    S->R = (double *)calloc(nl, sizeof(double));
    S->flip_site = (int64_t *)malloc(sizeof(int64_t) * nl);
    S->flip_old = (int8_t *)malloc(nl);
    S->flip_a = (int8_t *)malloc(nl);
    S->flip_fire = (uint8_t *)malloc(nl);
    S->perm = (uint32_t *)malloc(sizeof(uint32_t) * nl);
    if (!S->g.spin || !S->hist || !S->R || !S->flip_site || !S->flip_old || !S->flip_a || !S->flip_fire ||
        !S->perm) {
        free(S->g.spin); free(S->hist); free(S->R); free(S->flip_site);
        free(S->flip_old); free(S->flip_a); free(S->flip_fire); free(S->perm); free(S);
        return NULL;
    }
    init_spins(S->g.spin, S->N, p->seed, p->init);
    observables(&S->g, &S->M, &S->B);
    return S;
}

ORC_EXPORT void orc_sim_free(orc_sim *S) {
    if (!S) return;
    free(S->g.spin); free(S->hist); free(S->R); free(S->flip_site);
    free(S->flip_old); free(S->flip_a); free(S->flip_fire); free(S->perm);
    free(S);
}

static void flip_apply(orc_sim *S, int64_t site, int8_t old, int a) {
    S->g.spin[site] = (int8_t)(-old);
    S->M += -2 * (int64_t)old;
    S->B += 12 - 4 * (int64_t)a;
}

/* octant of the a-th active line for the drawn colour (R3 / R9) */
static int line_octant(const orc_sim *S, int colour, uint32_t a) {
    if (S->S != 2) return colour;
    uint32_t seen = 0;
    for (int s = 0; s < 8; ++s) {
        int parity = (s & 1) ^ ((s >> 1) & 1) ^ ((s >> 2) & 1);
        if (parity != colour) continue;
        if (seen == a) return s;
        ++seen;
    }
    return -1;
}

/* One spkMC cycle n (steps 1-6 with 4a/4b).  Returns the cycle increment dt. */
static double spkmc_cycle(orc_sim *S) {
    uint64_t n = S->n;
    uint32_t nlo = (uint32_t)n, nhi = (uint32_t)(n >> 32);
    uint32_t gw[4];
    /* step 4a and the step-5 draw: one stream shared by all domains */
    philox_words(S->p.seed, nlo, nhi, 0xFFFFFFFFu, 0xFFFFFFFFu, gw);
    int colour = (S->S == 8) ? (int)(gw[0] >> 29) : (S->S == 2) ? (int)(gw[0] >> 31) : 0;
    double ut = orc_uopen52(gw[2], gw[3]);
    const uint32_t nl = S->K * S->A; /* frequency lines (subdomains) of this cycle */

    /* step 1: frequency line of every active region (line f = A k + a) */
#pragma omp parallel for num_threads(orc_threads) if (orc_threads > 1) schedule(static)
    for (uint32_t f = 0; f < nl; ++f) {
        uint32_t k = f / S->A;
        int s = line_octant(S, colour, f % S->A);
        bin_region(S, k, s, &S->hist[(size_t)f * 14]);
        S->R[f] = line_total(&S->hist[(size_t)f * 14], S->r);
    }
    /* step 2: R_max (reading R4; scope 1 takes every octant of every colour;
     * scope 2 the fixed bound of R10) */
    double Rmax = 0.0;
    if (S->p.rmax_scope == 0) {
        for (uint32_t f = 0; f < nl; ++f)
            if (S->R[f] > Rmax) Rmax = S->R[f];
    } else if (S->p.rmax_scope == 1) {
#pragma omp parallel for num_threads(orc_threads) if (orc_threads > 1) schedule(static) reduction(max : Rmax)
        for (uint32_t k = 0; k < S->K; ++k)
            for (int c = 0; c < (S->S == 1 ? 1 : 8); ++c) {
                uint32_t h2[14];
                bin_region(S, k, c, h2);
                double Rc = line_total(h2, S->r);
                if (Rc > Rmax) Rmax = Rc;
            }
    } else {
        Rmax = S->Rbound;
        for (uint32_t f = 0; f < nl; ++f)
            if (S->R[f] > Rmax) S->check_fail++; /* cannot happen: R'_max bounds every line */
    }

    /* steps 3, 4, 4b: in every line an event with probability r / R_max */
    uint32_t nfire = 0;
    if (S->p.order == 0) {
        /* decide every line first (each line reads only its own region and
         * halo), then apply the flips in line order (step 6) */
        uint64_t fails = 0;
#pragma omp parallel for num_threads(orc_threads) if (orc_threads > 1) schedule(static) reduction(+ : nfire, fails)
        for (uint32_t f = 0; f < nl; ++f) {
            S->flip_fire[f] = 0;
            uint32_t k = f / S->A;
            int s = line_octant(S, colour, f % S->A);
            uint32_t dw[4];
            philox_words(S->p.seed, nlo, nhi, k, (uint32_t)s, dw);
            double u = orc_u53(dw[0], dw[1]);
            int32_t c;
            uint32_t j;
            if (!orc_select(&S->hist[(size_t)f * 14], S->r, Rmax, u, dw[2], &c, &j)) continue; /* null */
            int a = 0;
            int64_t site = find_site(S, k, s, c, j, &a);
            if (site < 0) {
                fails++;
                continue;
            }
            S->flip_fire[f] = 1;
            S->flip_site[f] = site;
            S->flip_old[f] = S->g.spin[site];
            S->flip_a[f] = (int8_t)a;
            ++nfire;
        }
        S->check_fail += fails;
        for (uint32_t f = 0; f < nl; ++f)
            if (S->flip_fire[f]) flip_apply(S, S->flip_site[f], S->flip_old[f], S->flip_a[f]);
    } else {
        /* apply each flip at once, in domain order (1) or a shuffled order (2) */
        for (uint32_t f = 0; f < nl; ++f) S->perm[f] = f;
        if (S->p.order == 2) {
            /* shuffled order: any permutation must give the same result */
            uint64_t st = 0x9E3779B97F4A7C15ull ^ n;
            for (uint32_t i = nl; i > 1; --i) {
                st = st * 6364136223846793005ull + 1442695040888963407ull;
                uint32_t jx = (uint32_t)((st >> 33) % i);
                uint32_t tmp = S->perm[i - 1];
                S->perm[i - 1] = S->perm[jx];
                S->perm[jx] = tmp;
            }
        }
        for (uint32_t ii = 0; ii < nl; ++ii) {
            uint32_t f = S->perm[ii];
            uint32_t k = f / S->A;
            int s = line_octant(S, colour, f % S->A);
            uint32_t dw[4];
            philox_words(S->p.seed, nlo, nhi, k, (uint32_t)s, dw);
            double u = orc_u53(dw[0], dw[1]);
            int32_t c;
            uint32_t j;
            const uint32_t *hk = &S->hist[(size_t)f * 14];
            /* flips already applied in this cycle must not have changed this
             * region or its halo: recompute and compare */
            uint32_t again[14];
            bin_region(S, k, s, again);
            if (memcmp(again, hk, sizeof(again)) != 0) S->check_fail++;
            if (!orc_select(hk, S->r, Rmax, u, dw[2], &c, &j)) continue; /* null event */
            int a = 0;
            int64_t site = find_site(S, k, s, c, j, &a);
            if (site < 0) {
                S->check_fail++;
                continue;
            }
            flip_apply(S, site, S->g.spin[site], a);
            ++nfire;
        }
    }

    /* step 5: common time increment (reading R5) */
    double dt = -log(ut) / ((double)S->S * Rmax);
    S->t = S->t + dt;
    S->fired += nfire;
    S->nulls += (uint64_t)nl - nfire;
    S->n = n + 1;
    if (S->p.check) {
        int64_t M, B;
        observables(&S->g, &M, &B);
        if (M != S->M || B != S->B) S->check_fail++;
    }
    return dt;
}

static void fill_record(const orc_sim *S, orc_record *r) {
    r->cycle = S->n;
    r->fired = S->fired;
    r->nulls = S->nulls;
    r->t = S->t;
    r->M = S->M;
    r->B = S->B;
}

/* Run ncycles; every obs_every cycles (counted by the absolute cycle number)
 * append a record of the state after that cycle. */
ORC_EXPORT int orc_sim_run(orc_sim *S, uint64_t ncycles, uint32_t obs_every, orc_record *rec,
                           uint64_t cap, uint64_t *nrec) {
    uint64_t nr = 0;
    for (uint64_t i = 0; i < ncycles; ++i) {
        spkmc_cycle(S);
        if (obs_every && (S->n % obs_every) == 0) {
            if (rec && nr < cap) fill_record(S, &rec[nr]);
            ++nr;
        }
    }
    if (nrec) *nrec = nr;
    return 0;
}

ORC_EXPORT void orc_sim_state(const orc_sim *S, orc_record *out) { fill_record(S, out); }
ORC_EXPORT uint64_t orc_sim_check_failures(const orc_sim *S) { return S->check_fail; }
ORC_EXPORT void orc_sim_get_spins(const orc_sim *S, int8_t *out) { memcpy(out, S->g.spin, (size_t)S->N); }
ORC_EXPORT double orc_sim_rate(const orc_sim *S, int c) { return S->r[c]; }
ORC_EXPORT double orc_sim_rbound(const orc_sim *S) { return S->Rbound; }

/* Replace the spins (values must be +-1) and recompute M, B; counters and the
 * clock are set from the arguments (a resumed state). */
ORC_EXPORT int orc_sim_set_state(orc_sim *S, const int8_t *in, uint64_t cycle, uint64_t fired,
                                 uint64_t nulls, double t) {
    for (int64_t i = 0; i < S->N; ++i)
        if (in[i] != 1 && in[i] != -1) return -1;
    memcpy(S->g.spin, in, (size_t)S->N);
    observables(&S->g, &S->M, &S->B);
    S->n = cycle;
    S->fired = fired;
    S->nulls = nulls;
    S->t = t;
    return 0;
}

/* Histogram of the octant (k, s) of the current state (for tests). */
ORC_EXPORT void orc_sim_octant_hist(const orc_sim *S, uint32_t k, int32_t s, uint32_t out[14]) {
    bin_region(S, k, s, out);
}

/* Sample M and B on a fixed time grid: the value at time t_m is the state
 * after the last cycle whose clock is <= t_m.  The grid must be increasing.
 * Stops after max_cycles; returns the number of grid points filled. */
ORC_EXPORT uint64_t orc_sim_run_grid(orc_sim *S, const double *grid, uint64_t ngrid, int64_t *Mo,
                                     int64_t *Bo, uint64_t max_cycles) {
    uint64_t m = 0, c = 0;
    while (m < ngrid && grid[m] < S->t) { Mo[m] = S->M; Bo[m] = S->B; ++m; }
    while (m < ngrid && c < max_cycles) {
        int64_t M0 = S->M, B0 = S->B;
        spkmc_cycle(S);
        ++c;
        /* state (M0,B0) held on [t0, t_new) */
        while (m < ngrid && grid[m] < S->t) { Mo[m] = M0; Bo[m] = B0; ++m; }
    }
    return m;
}

/* Time-weighted accumulation over ncycles: tw[0] += dt, tw[1] += E dt,
 * tw[2] += |M| dt, tw[3] += M^2 dt, where (E, M) is the state held during dt.
 * If hist is given (N <= 16), hist[state] += dt with state bit i = (s_i > 0). */
ORC_EXPORT void orc_sim_run_tw(orc_sim *S, uint64_t ncycles, double tw[4], double *hist) {
    for (uint64_t i = 0; i < ncycles; ++i) {
        int64_t M0 = S->M, B0 = S->B;
        uint32_t code = 0;
        if (hist && S->N <= 16)
            for (int64_t q = 0; q < S->N; ++q) code |= (uint32_t)(S->g.spin[q] > 0) << q;
        double dt = spkmc_cycle(S);
        double E = -S->p.J * (double)B0 - S->p.H * (double)M0;
        tw[0] += dt;
        tw[1] += E * dt;
        tw[2] += (double)(M0 < 0 ? -M0 : M0) * dt;
        tw[3] += (double)M0 * (double)M0 * dt;
        if (hist && S->N <= 16) hist[code] += dt;
    }
}

/* ------------------------------------------------------------------------- */
/* Serial BKL / n-fold way (the serial reference of Sec. 4).                  */
/* Classes over all N sites; R_tot = sum_c n_c r_c (fixed order); the class   */
/* from u R_tot, the site uniform inside the class (per-class site lists with */
/* swap-remove), or the j-th site of the class in canonical lattice order     */
/* (canonical mode); dt = -ln(u_t) / R_tot.                                   */
/* Draws of event e: counter (e_lo, e_hi, 0xFFFFFFFD, 0): u = u53(w0, w1),    */
/* u_t = uopen52(w2, w3); counter (e_lo, e_hi, 0xFFFFFFFD, 1): w0 = site word.*/
/* draw_mode 1 instead consumes the spkMC streams of a one-domain,            */
/* one-colour run (the identity test).                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    orc_params p;
    int L;
    int64_t N;
    double r[14];
    lattice g;
    int8_t *cls;      /* class of every site */
    int64_t *list;    /* 14 lists of capacity N, concatenated */
    int64_t *pos;     /* position of each site in its class list */
    uint32_t cnt[14];
    int canonical, draw_mode;
    uint64_t e;
    double t;
    int64_t M, B;
} orc_bkl;

static int64_t bkl_index(const orc_bkl *K, int x, int y, int z) {
    return (int64_t)x + (int64_t)K->L * ((int64_t)y + (int64_t)K->L * z);
}

static void bkl_remove(orc_bkl *K, int64_t i) {
    int c = K->cls[i];
    int64_t p = K->pos[i];
    int64_t last = K->list[(int64_t)c * K->N + K->cnt[c] - 1];
    K->list[(int64_t)c * K->N + p] = last;
    K->pos[last] = p;
    K->cnt[c]--;
}
static void bkl_insert(orc_bkl *K, int64_t i, int c) {
    K->cls[i] = (int8_t)c;
    K->pos[i] = K->cnt[c];
    K->list[(int64_t)c * K->N + K->cnt[c]] = i;
    K->cnt[c]++;
}

ORC_EXPORT orc_bkl *orc_bkl_new(const orc_params *p, int32_t canonical, int32_t draw_mode) {
    if (!p || p->L < 2) return NULL;
    orc_bkl *K = (orc_bkl *)calloc(1, sizeof(orc_bkl));
    if (!K) return NULL;
    K->p = *p;
    K->L = p->L;
    K->N = (int64_t)p->L * p->L * p->L;
    K->canonical = canonical;
    K->draw_mode = draw_mode;
    if (orc_rate_table(p->J, p->H, p->T, p->rates, K->r) != 0) { free(K); return NULL; }
    K->g.L = p->L;
    K->g.spin = (int8_t *)malloc((size_t)K->N);
    K->cls = (int8_t *)malloc((size_t)K->N);
    K->list = (int64_t *)malloc(sizeof(int64_t) * (size_t)K->N * 14);
    K->pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)K->N);
    if (!K->g.spin || !K->cls || !K->list || !K->pos) {
        free(K->g.spin); free(K->cls); free(K->list); free(K->pos); free(K);
        return NULL;
    }
    init_spins(K->g.spin, K->N, p->seed, p->init);
    observables(&K->g, &K->M, &K->B);
    for (int z = 0; z < K->L; ++z)
        for (int y = 0; y < K->L; ++y)
            for (int x = 0; x < K->L; ++x) bkl_insert(K, bkl_index(K, x, y, z), site_class(&K->g, x, y, z));
    return K;
}

ORC_EXPORT void orc_bkl_free(orc_bkl *K) {
    if (!K) return;
    free(K->g.spin); free(K->cls); free(K->list); free(K->pos); free(K);
}

/* one BKL event; returns dt */
static double bkl_event(orc_bkl *K) {
    double u, ut;
    uint32_t sw;
    if (K->draw_mode == 1) {
        uint32_t gw[4], dw[4];
        philox_words(K->p.seed, (uint32_t)K->e, (uint32_t)(K->e >> 32), 0xFFFFFFFFu, 0xFFFFFFFFu, gw);
        philox_words(K->p.seed, (uint32_t)K->e, (uint32_t)(K->e >> 32), 0u, 0u, dw);
        u = orc_u53(dw[0], dw[1]);
        sw = dw[2];
        ut = orc_uopen52(gw[2], gw[3]);
    } else {
        uint32_t w[4], w2[4];
        philox_words(K->p.seed, (uint32_t)K->e, (uint32_t)(K->e >> 32), 0xFFFFFFFDu, 0u, w);
        philox_words(K->p.seed, (uint32_t)K->e, (uint32_t)(K->e >> 32), 0xFFFFFFFDu, 1u, w2);
        u = orc_u53(w[0], w[1]);
        ut = orc_uopen52(w[2], w[3]);
        sw = w2[0];
    }
    double Rtot = line_total(K->cnt, K->r);
    int32_t c;
    uint32_t j;
    /* with R_max = R_tot there is no null segment */
    if (!orc_select(K->cnt, K->r, Rtot, u, sw, &c, &j)) {
        /* u R_tot rounded up to R_tot: take the last populated class */
        for (c = 13; c >= 0 && K->cnt[c] == 0; --c) {}
        j = orc_idx(sw, K->cnt[c]);
    }
    int64_t site;
    if (K->canonical) {
        uint32_t seen = 0;
        site = -1;
        for (int64_t i = 0; i < K->N; ++i)
            if (K->cls[i] == c) {
                if (seen == j) { site = i; break; }
                ++seen;
            }
    } else {
        site = K->list[(int64_t)c * K->N + j];
    }
    int x = (int)(site % K->L), y = (int)((site / K->L) % K->L), z = (int)(site / ((int64_t)K->L * K->L));
    int8_t old = K->g.spin[site];
    int a = c % 7;
    K->g.spin[site] = (int8_t)(-old);
    K->M += -2 * (int64_t)old;
    K->B += 12 - 4 * (int64_t)a;
    /* classes of the flipped site and its 6 neighbours change */
    int L = K->L;
    int xs[7] = {x, wrap_dec(x, L), wrap_inc(x, L), x, x, x, x};
    int ys[7] = {y, y, y, wrap_dec(y, L), wrap_inc(y, L), y, y};
    int zs[7] = {z, z, z, z, z, wrap_dec(z, L), wrap_inc(z, L)};
    for (int q = 0; q < 7; ++q) {
        int64_t i = bkl_index(K, xs[q], ys[q], zs[q]);
        int nc = site_class(&K->g, xs[q], ys[q], zs[q]);
        if (nc != K->cls[i]) {
            bkl_remove(K, i);
            bkl_insert(K, i, nc);
        }
    }
    double dt = -log(ut) / Rtot;
    K->t = K->t + dt;
    K->e++;
    return dt;
}

ORC_EXPORT void orc_bkl_run(orc_bkl *K, uint64_t nevents) {
    for (uint64_t i = 0; i < nevents; ++i) bkl_event(K);
}

ORC_EXPORT void orc_bkl_state(const orc_bkl *K, orc_record *out) {
    out->cycle = K->e;
    out->fired = K->e;
    out->nulls = 0;
    out->t = K->t;
    out->M = K->M;
    out->B = K->B;
}
ORC_EXPORT void orc_bkl_get_spins(const orc_bkl *K, int8_t *out) { memcpy(out, K->g.spin, (size_t)K->N); }
ORC_EXPORT void orc_bkl_counts(const orc_bkl *K, uint32_t out[14]) { memcpy(out, K->cnt, sizeof(K->cnt)); }

/* time grid sampling, as orc_sim_run_grid */
ORC_EXPORT uint64_t orc_bkl_run_grid(orc_bkl *K, const double *grid, uint64_t ngrid, int64_t *Mo,
                                     int64_t *Bo, uint64_t max_events) {
    uint64_t m = 0, c = 0;
    while (m < ngrid && grid[m] < K->t) { Mo[m] = K->M; Bo[m] = K->B; ++m; }
    while (m < ngrid && c < max_events) {
        int64_t M0 = K->M, B0 = K->B;
        bkl_event(K);
        ++c;
        while (m < ngrid && grid[m] < K->t) { Mo[m] = M0; Bo[m] = B0; ++m; }
    }
    return m;
}

ORC_EXPORT void orc_bkl_run_tw(orc_bkl *K, uint64_t nevents, double tw[4], double *hist) {
    for (uint64_t i = 0; i < nevents; ++i) {
        int64_t M0 = K->M, B0 = K->B;
        uint32_t code = 0;
        if (hist && K->N <= 16)
            for (int64_t q = 0; q < K->N; ++q) code |= (uint32_t)(K->g.spin[q] > 0) << q;
        double dt = bkl_event(K);
        double E = -K->p.J * (double)B0 - K->p.H * (double)M0;
        tw[0] += dt;
        tw[1] += E * dt;
        tw[2] += (double)(M0 < 0 ? -M0 : M0) * dt;
        tw[3] += (double)M0 * (double)M0 * dt;
        if (hist && K->N <= 16) hist[code] += dt;
    }
}

/* Observables of an arbitrary +-1 lattice (for tests). */
ORC_EXPORT void orc_observables(const int8_t *spin, int32_t L, int64_t *M, int64_t *B) {
    lattice g;
    g.L = L;
    g.spin = (int8_t *)spin;
    observables(&g, M, B);
}
/* Class of one site of an arbitrary lattice (for tests). */
ORC_EXPORT int32_t orc_site_class(const int8_t *spin, int32_t L, int32_t x, int32_t y, int32_t z) {
    lattice g;
    g.L = L;
    g.spin = (int8_t *)spin;
    return site_class(&g, x, y, z);
}
/* The initial spins the seed gives (for tests). */
ORC_EXPORT void orc_init_spins(int8_t *spin, int64_t N, uint64_t seed, int32_t init) {
    init_spins(spin, N, seed, init);
}
