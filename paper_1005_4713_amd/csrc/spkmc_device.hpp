// spkmc_device.hpp -- device-side state, geometry and random numbers of the
// gfx950 spkMC library (host and device code of the library include it; the
// CPU oracle does not).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spkmc.h"

#pragma clang fp contract(off)

namespace spkmc {

// Device-resident counters of one lattice, at offset 0 of the caller's buffer.
struct alignas(256) DevState {
    uint64_t cycle;        // cycles completed
    uint64_t fired;        // non-null events
    uint64_t nulls;        // null events
    double t;              // simulated time
    int64_t M;             // sum of spins
    int64_t B;             // sum of nearest-neighbour bond products (each bond once)
    uint64_t rec_count;    // records written (ring index = rec_count % record_cap)
    uint32_t error;        // non-zero: a device-side wait gave up (see kErr*)
    uint32_t pad0;
    uint64_t rmax[4];      // per-cycle R_max slots: FP64 bit patterns (R >= 0, so the
                           // unsigned order of the bits is the order of the values)
    uint64_t acc_fired[4]; // per-cycle partial sums of the select phase
    int64_t acc_dM[4];
    int64_t acc_dB[4];
    uint64_t pad1[8];
};
static_assert(sizeof(DevState) == 256, "DevState must stay 256 bytes");

enum : uint32_t { kErrBarrierTimeout = 1, kErrFlagTimeout = 2, kErrSelect = 4, kErrHist = 8 };

// Geometry and buffer addresses, passed to every kernel by value.
struct Geom {
    int32_t L, d, h, nd;   // lattice edge, domain edge, octant edge, domains per edge
    int32_t layout;        // SPKMC_LAYOUT_*
    uint32_t K;            // domains
    uint64_t N;            // sites
    uint32_t h2, h3;       // h^2, h^3
    uint32_t wpo;          // PACKED: 32-bit words per octant (h^3 / 32)
    uint32_t fwpo;         // PACKED: halo-copy words per octant (6 h^2 / 32)
    uint32_t rec_cap;
    uint32_t variant;      // SPKMC_VARIANT_* bits
    uint64_t seed;
    DevState *st;
    spkmc_record *rec;
    double *Rk;            // K
    uint32_t *hist;        // K x 16 (14 used)
    uint64_t *flip;        // K flip records
    uint64_t *sync;        // persistent engine: R_max slots, flags, record partials (9 G words)
    uint64_t *dh;          // PACKED: class changes pushed across workgroups, K x 8 octants x 2 spins
    uint32_t *sc;          // PACKED, h = 16: per octant the class counts of its four 4-plane slabs (28 words)
    int8_t *spin8;         // INT8 spins
    uint32_t *A;           // PACKED spins, octant-major, canonical order inside an octant
    uint32_t *F;           // PACKED halo copies: per octant its halo faces x below, x above, y below,
                           // y above, z below, z above (h^2 bits each)
    double r[14];          // rate table
    double rbound;         // R'_max = n_k max_c r_c (RMAX_BOUND)
    uint32_t lpd;          // frequency lines per domain and cycle: 1, or 4 (TWO_COLOURS)
    uint32_t pad2;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): two 32x32 -> 64-bit products per round,
// key advanced by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key) {
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// [0, 1) with 53 random bits
__host__ __device__ inline double unit53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}
// (0, 1): a 52-bit integer plus one half, over 2^52
__host__ __device__ inline double unit_open52(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 4503599627370496.0);
}
__host__ __device__ inline uint32_t mul_index(uint32_t w, uint32_t n) {
    return (uint32_t)(((uint64_t)w * n) >> 32);
}

// The per-cycle draw shared by every domain: colour (top 3 bits of the first
// word; with two colours its top bit) and the clock uniform.
struct CycleDraw {
    int colour;
    double ut;
};
__host__ __device__ inline CycleDraw cycle_draw(uint64_t seed, uint64_t n, bool two_colours = false) {
    U4 w = philox10((uint32_t)n, (uint32_t)(n >> 32), 0xFFFFFFFFu, 0xFFFFFFFFu, seed);
    return CycleDraw{(int)(w.x >> (two_colours ? 31 : 29)), unit_open52(w.z, w.w)};
}
// Octant of the i-th frequency line (i < 4) of colour c with two colours: the
// octants whose sx + sy + sz has parity c, in increasing order.
__host__ __device__ inline int two_colour_octant(int c, uint32_t i) {
    return c ? (int)((0x7421u >> (4 * i)) & 15u) : (int)((0x6530u >> (4 * i)) & 15u);
}

// Fixed-order FP64 frequency line: separate multiply and add, classes 0..13.
__device__ inline double line_total(const uint32_t *cnt, const double *r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 14; ++c) {
        double term = (double)cnt[c] * r[c];
        acc = acc + term;
    }
    return acc;
}
// Class chosen by target = u R_max on the same running sums; -1 = null event.
__device__ inline int line_select(const uint32_t *cnt, const double *r, double target) {
    double acc = 0.0;
    int chosen = -1;
#pragma unroll
    for (int c = 0; c < 14; ++c) {
        double term = (double)cnt[c] * r[c];
        acc = acc + term;
        if (chosen < 0 && target < acc) chosen = c;
    }
    return chosen;
}

__device__ inline double bits_to_double(uint64_t b) { return __longlong_as_double((long long)b); }
__device__ inline uint64_t double_to_bits(double v) { return (uint64_t)__double_as_longlong(v); }

// Step 5 and the bookkeeping of cycle n on the per-cycle engine (one thread,
// after every workgroup's selection and flips): the clock, the counters from
// the partials, the observation record; the per-cycle accumulators reset.
__device__ inline void finalize_cycle(const Geom &g, uint64_t n, uint32_t obs_every) {
    DevState *st = g.st;
    const bool two = g.lpd == 4;
    const CycleDraw cd = cycle_draw(g.seed, n, two);
    const double Rmax = (g.variant & SPKMC_VARIANT_RMAX_BOUND) ? g.rbound : bits_to_double(st->rmax[0]);
    const double dt = -log(cd.ut) / ((two ? 2.0 : 8.0) * Rmax);
    st->t = st->t + dt;
    const uint64_t f = st->acc_fired[0];
    st->fired += f;
    st->nulls += (uint64_t)g.K * g.lpd - f;
    st->M += st->acc_dM[0];
    st->B += st->acc_dB[0];
    st->acc_fired[0] = 0;
    st->acc_dM[0] = 0;
    st->acc_dB[0] = 0;
    st->rmax[0] = 0;
    st->cycle = n + 1;
    if (obs_every && ((n + 1) % obs_every) == 0 && g.rec_cap) {
        spkmc_record r;
        r.cycle = n + 1;
        r.fired = st->fired;
        r.nulls = st->nulls;
        r.t = st->t;
        r.M = st->M;
        r.B = st->B;
        g.rec[st->rec_count % g.rec_cap] = r;
        st->rec_count += 1;
    }
}

// ---------------------------------------------------------------------------
// Site addressing.
// ---------------------------------------------------------------------------
struct OctAddr {
    uint32_t k;
    int s;
    uint32_t q;
};
__device__ inline OctAddr octant_of(const Geom &g, int x, int y, int z) {
    int kx = x / g.d, ky = y / g.d, kz = z / g.d;
    int rx = x - kx * g.d, ry = y - ky * g.d, rz = z - kz * g.d;
    int sx = rx >= g.h, sy = ry >= g.h, sz = rz >= g.h;
    int lx = rx - sx * g.h, ly = ry - sy * g.h, lz = rz - sz * g.h;
    OctAddr a;
    a.k = (uint32_t)kx + (uint32_t)g.nd * ((uint32_t)ky + (uint32_t)g.nd * (uint32_t)kz);
    a.s = sx | (sy << 1) | (sz << 2);
    a.q = (uint32_t)lx + (uint32_t)g.h * ((uint32_t)ly + (uint32_t)g.h * (uint32_t)lz);
    return a;
}

struct Int8Spins {
    __device__ static inline int get(const Geom &g, int x, int y, int z) {
        return g.spin8[(int64_t)x + (int64_t)g.L * ((int64_t)y + (int64_t)g.L * z)];
    }
};
struct PackedSpins {
    __device__ static inline int get(const Geom &g, int x, int y, int z) {
        OctAddr a = octant_of(g, x, y, z);
        uint64_t bit = ((uint64_t)a.k * 8 + (uint64_t)a.s) * g.h3 + a.q;
        return ((g.A[bit >> 5] >> (bit & 31)) & 1u) ? 1 : -1;
    }
};

template <class S>
__device__ inline int aligned_count(const Geom &g, int x, int y, int z, int s) {
    int L = g.L;
    int xm = x ? x - 1 : L - 1, xp = x + 1 == L ? 0 : x + 1;
    int ym = y ? y - 1 : L - 1, yp = y + 1 == L ? 0 : y + 1;
    int zm = z ? z - 1 : L - 1, zp = z + 1 == L ? 0 : z + 1;
    return (S::get(g, xm, y, z) == s) + (S::get(g, xp, y, z) == s) + (S::get(g, x, ym, z) == s) +
           (S::get(g, x, yp, z) == s) + (S::get(g, x, y, zm) == s) + (S::get(g, x, y, zp) == s);
}

// Origin of octant (k, s).
__device__ inline void octant_origin(const Geom &g, uint32_t k, int s, int &ox, int &oy, int &oz) {
    uint32_t nd = (uint32_t)g.nd;
    int kx = (int)(k % nd), ky = (int)((k / nd) % nd), kz = (int)(k / (nd * nd));
    ox = kx * g.d + (s & 1) * g.h;
    oy = ky * g.d + ((s >> 1) & 1) * g.h;
    oz = kz * g.d + ((s >> 2) & 1) * g.h;
}

}  // namespace spkmc
