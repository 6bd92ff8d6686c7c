// kernels_slab.hip -- the slab engine of the gfx950 spkMC library (PACKED,
// octant edge 16): the class counts of every octant, per slab of four z-planes,
// kept in device memory and moved by every flip; the persistent kernel
// k_slab<ALL> and the per-cycle slab kernels (persistent_common.hpp holds the
// shared binning, selection and flip code).
#include <string>

#include "api_internal.hpp"
#include "persistent_common.hpp"

namespace spkmc {

// ---------------------------------------------------------------------------
// Slab engine (PACKED, octant edge 16, eight colours, R_max exchanged).  The
// class counts of every octant live in device memory, split over its four
// slabs of four z-planes (28 words per octant: class c, slabs 2i and 2i + 1 as
// the 16-bit halves of word 2c + i).  A cycle reads the counts of the active
// octants instead of binning them (step 1), takes the frequency lines and
// R_max from them (steps 1 and 2), and locates the selected site (step 4b) by
// classifying only the slab whose running count of the chosen class passes the
// site's rank.  Each flip moves the flipped site and its six neighbours between
// classes (step 6): the counts of the active octant in LDS, written back at the
// end of the cycle (no other domain's flip reaches an active octant), those of
// the face-adjacent octants by device atomics.
// ---------------------------------------------------------------------------
constexpr int kSlabRows = 32, kSlabPasses = 4, kSlabBlock = kSlabRows * 16;
constexpr uint32_t kSlabDomains = kSlabRows * kSlabPasses;  // domains of one workgroup
constexpr uint32_t kSlabWords = 28;                         // slab count words per octant
// per domain in LDS: the 128 words of the active octant (plane z: words 8z ..
// 8z + 7, word w holding rows 2w and 2w + 1), then its halo faces x below, x
// above, y below, y above, z below, z above (8 words each, the face-copy layout)
constexpr int kOctLds = 176;
constexpr int kFxm = 128, kFxp = 136, kFym = 144, kFyp = 152, kFzm = 160, kFzp = 168;

struct SlabShared {
    double r[14];
    alignas(16) uint32_t oct[kSlabDomains][kOctLds];    // active octants and their halos
    uint32_t sc[kSlabDomains][kSlabWords];  // slab counts of the active octants
    uint16_t cnt[kSlabDomains][8][14];      // class counts (the active octant; every octant for the all-octant R_max)
    double acc[kSlabDomains][14];           // running FP64 sums of the frequency lines
    double rk[kSlabDomains];
    alignas(16) uint32_t zbuf[kSlabRows][kRowHalo];     // binning at launch start: halo faces per row
    uint32_t nbdom[kSlabDomains][6];
    uint32_t dco[kSlabDomains];             // domain coordinates kx | ky << 10 | kz << 20
    uint32_t selq[kSlabDomains];
    double rpred[8];
    double rmax;
    int abort;
    uint32_t nbr_bits[6][kMaxGrid / 32];
    uint32_t nbr_cnt[6];
    uint32_t nbr[6][kMaxNbr];
    long long red[3][16];
    uint32_t pend_head, pend_tail;
    uint64_t pend_cycle[kRecBanks];
    double pend_t[kRecBanks];
    uint32_t pend_bank[kRecBanks];
};

__device__ __forceinline__ void st32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin (1 = up) of the active octant at local (x, y, z), each in [-1, 16] and
// at most one outside [0, 16): the octant's words or one of its halo faces.
__device__ __forceinline__ uint32_t slab_spin(const uint32_t *o, int x, int y, int z) {
    int base = 0, b = x + 16 * y + 256 * z;
    if ((unsigned)x > 15u) base = x < 0 ? kFxm : kFxp, b = y + 16 * z;
    if ((unsigned)y > 15u) base = y < 0 ? kFym : kFyp, b = x + 16 * z;
    if ((unsigned)z > 15u) base = z < 0 ? kFzm : kFzp, b = x + 16 * y;
    return (o[base + (b >> 5)] >> (b & 31)) & 1u;
}
// Class of the site at octant-local (x, y, z) inside the octant, from the words
// and halo in LDS.
__device__ __forceinline__ int slab_class_lds(const uint32_t *o, int x, int y, int z) {
    const uint32_t nup = slab_spin(o, x - 1, y, z) + slab_spin(o, x + 1, y, z) + slab_spin(o, x, y - 1, z) +
                         slab_spin(o, x, y + 1, z) + slab_spin(o, x, y, z - 1) + slab_spin(o, x, y, z + 1);
    return site_class(slab_spin(o, x, y, z), (int)nup);
}
// A site of slab b leaves class c_old for c_new: the slab counts of its octant.
__device__ __forceinline__ void slab_move_lds(uint32_t *sc, int c_old, int c_new, int b) {
    const int sh = 16 * (b & 1);
    atomicAdd(&sc[2 * c_old + (b >> 1)], 0u - (1u << sh));
    atomicAdd(&sc[2 * c_new + (b >> 1)], 1u << sh);
}
__device__ __forceinline__ void slab_move_dev(uint32_t *sc, int c_old, int c_new, int b) {
    const int sh = 16 * (b & 1);
    (void)__hip_atomic_fetch_add(&sc[2 * c_old + (b >> 1)], 0u - (1u << sh), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    (void)__hip_atomic_fetch_add(&sc[2 * c_new + (b >> 1)], 1u << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The event of the row of domain ld for class cs (-1: none), written into its
// selection slot as (cs << 12) | q, or kNoEvent.  The site is the j-th of class
// cs in canonical order (j from uz): the slab is the one whose running count of
// the class passes j; lane l of the row classifies words 2 (l & 3) and
// 2 (l & 3) + 1 of plane 4 slab + l / 4 of that slab, so the lanes run in
// canonical order.  Every lane of the row takes part.
__device__ __forceinline__ void slab_select(const uint32_t *sc, const uint32_t *o, int cs, uint32_t uz, int l,
                                            uint32_t *slot, DevState *st) {
    if (l == 0) *slot = kNoEvent;
    const int c = cs >= 0 ? cs : 0;
    const uint32_t v0 = sc[2 * c], v1 = sc[2 * c + 1];
    const uint32_t e1 = v0 & 0xFFFFu, e2 = e1 + (v0 >> 16), e3 = e2 + (v1 & 0xFFFFu), ncs = e3 + (v1 >> 16);
    const uint32_t j = cs >= 0 ? mul_index(uz, ncs) : 0u;
    const uint32_t b = (j >= e1 ? 1u : 0u) + (j >= e2 ? 1u : 0u) + (j >= e3 ? 1u : 0u);
    const uint32_t rank = j - (b == 0 ? 0u : b == 1 ? e1 : b == 2 ? e2 : e3);
    const int pz = 4 * (int)b + (l >> 2), wi = 2 * (l & 3);
    const uint32_t wa = o[8 * pz + wi], wb = o[8 * pz + wi + 1];
    // y neighbours: row 2 wi - 1 (the previous word, or the face below) and row
    // 2 wi + 4 (the word after next, or the face above); a face row of plane pz
    // is half-word pz & 1 of face word pz / 2
    const int fh = 16 * (pz & 1);
    const uint32_t prev = wi == 0 ? ((o[kFym + (pz >> 1)] >> fh) & 0xFFFFu) << 16 : o[8 * pz + wi - 1];
    const uint32_t next = wi == 6 ? (o[kFyp + (pz >> 1)] >> fh) & 0xFFFFu : o[8 * pz + wi + 2];
    // z neighbours: planes pz -+ 1, or the z faces (the same word layout as a plane)
    const int zm = pz == 0 ? kFzm + wi : 8 * (pz - 1) + wi, zp = pz == 15 ? kFzp + wi : 8 * (pz + 1) + wi;
    const uint32_t zma = o[zm], zmb = o[zm + 1], zpa = o[zp], zpb = o[zp + 1];
    // x neighbours: the x faces hold rows 2 wi .. 2 wi + 3 of plane pz at bits fh + 2 wi ..
    const uint32_t xm = o[kFxm + (pz >> 1)] >> (fh + 2 * wi), xp = o[kFxp + (pz >> 1)] >> (fh + 2 * wi);
    const uint32_t Tma = (xm & 1u) | ((xm & 2u) << 15), Tmb = ((xm >> 2) & 1u) | ((xm & 8u) << 13);
    const uint32_t Tpa = ((xp & 1u) << 15) | ((xp & 2u) << 30), Tpb = ((xp & 4u) << 13) | ((xp & 8u) << 28);
    // class cs as (spin, n_up pattern), as in select_site
    const int up = cs >= 7, v = up ? cs - 7 : 6 - cs;
    const uint32_t ps = up ? 0xFFFFFFFFu : 0u, p0 = (v & 1) ? 0xFFFFFFFFu : 0u;
    const uint32_t p1 = (v & 2) ? 0xFFFFFFFFu : 0u, p2 = (v & 4) ? 0xFFFFFFFFu : 0u;
    uint32_t mk[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const uint32_t w = i ? wb : wa;
        const uint32_t nxm = bop<kSelAC_BnC>(w << 1, i ? Tmb : Tma, 0xFFFEFFFEu);
        const uint32_t nxp = bop<kSelAC_BnC>(w >> 1, i ? Tpb : Tpa, 0x7FFF7FFFu);
        const uint32_t nym = i ? align_hi(wb, wa, 16) : align_hi(wa, prev, 16);
        const uint32_t nyp = i ? align_hi(next, wb, 16) : align_hi(wb, wa, 16);
        uint32_t o0, o1, o2;
        count6(nxm, nxp, nym, nyp, i ? zmb : zma, i ? zpb : zpa, o0, o1, o2);
        uint32_t d = w ^ ps;
        d = bop<kXorOr>(o0, p0, d);
        d = bop<kXorOr>(o1, p1, d);
        mk[i] = bop<kXorNor>(o2, p2, d);
    }
    const uint32_t ca = (uint32_t)__builtin_popcount(mk[0]);
    const uint32_t tot = bcnt_acc(mk[1], ca);
    const uint32_t incl = row_scan(tot), excl = incl - tot;
    if (cs >= 0 && l == 15 && rank >= incl) atomicOr(&st->error, kErrSelect);  // counts disagree with the spins
    if (cs >= 0 && rank >= excl && rank < incl) {
        const uint32_t r0 = rank - excl;
        const bool first = r0 < ca;
        const uint32_t bit = (uint32_t)nth_set_bit(first ? mk[0] : mk[1], first ? r0 : r0 - ca);
        const uint32_t q = (uint32_t)(256 * pz) + 32u * (uint32_t)(wi + (first ? 0 : 1)) + bit;
        *slot = ((uint32_t)cs << 12) | q;
    }
}

// Bin octant o of every domain of the workgroup into its slab counts in device
// memory: the 13 moments of each plane (lane), summed over the slab's four
// lanes, give the slab's histogram.
template <class SH>
__device__ __forceinline__ void slab_bin_octant(const Geom &g, uint32_t kbase, uint32_t nvalid, int o, SH &sh) {
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
#pragma unroll 1
    for (int pp = 0; pp < kSlabPasses; ++pp) {
        const uint32_t ld = (uint32_t)(pp * kSlabRows + row);
        const bool valid = ld < nvalid;
        Raw<16> raw;
        Planes<16> pl;
        load_octant<16>(g, kbase + ld, o, valid, l, sh.nbdom[valid ? ld : 0], raw);
        uint32_t m[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) m[i] = 0;
        compute16<true>(raw, valid, l, sh.zbuf[row], pl, m);
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            m[i] += dpp0<kRowShr1>(m[i]);
            m[i] += dpp0<kRowShr2>(m[i]);  // lane 4 b + 3: the sum over slab b
        }
        uint32_t hc[14];
        hist_from_moments(m, 1024u, hc);
        // lanes 7 and 15 write slabs 0, 1 and 2, 3 of every class
        uint32_t *dst = g.sc + ((uint64_t)(kbase + ld) * 8 + (uint32_t)o) * kSlabWords + (l >> 3);
#pragma unroll
        for (int c = 0; c < 14; ++c) {
            const uint32_t lo = dpp0<kRowShr4>(hc[c]);  // lane 4 b + 3 -> 4 b + 7
            if (valid && (l & 7) == 7) st32(dst + 2 * c, lo | (hc[c] << 16));
        }
    }
}

// Part `part` of the flip f = (cs << 12) | q of octant (k, so): part 0 flips the
// site (its spin word and halo copies) and moves its class; parts 1..3 move the
// classes of its two neighbours along axis part - 1.  A neighbour inside the
// octant takes its class from the octant and halo in LDS (o; the flipped site
// still reads its old spin there) and moves in the octant's counts in LDS (sc);
// one across a face reads its own neighbours from memory (none of them flips in
// the same cycle) and moves in that octant's counts by device atomics.  dco_k:
// the coordinates of domain k (kx | ky << 10 | kz << 20).
__device__ __forceinline__ void slab_flip_part(const Geom &g, const uint32_t *o, uint32_t *sc, uint32_t dco_k,
                                               const uint32_t *nb, uint32_t k, int so, uint32_t f, int part, long long &F,
                                               long long &dM, long long &dB) {
    const int cs = (int)(f >> 12);
    const uint32_t q = f & 0xFFFu;
    const int lx = (int)(q & 15u), ly = (int)((q >> 4) & 15u), lz = (int)(q >> 8);
    const uint32_t up = cs >= 7;
    if (part == 0) {
        slab_move_lds(sc, cs, site_class(!up, up ? cs - 7 : 6 - cs), lz >> 2);
        flip_site<16>(g, k, so, q, nb);
        F += 1;
        dM += up ? -2 : 2;
        dB += 12 - 4 * (long long)(cs % 7);
    } else {
        // axis part - 1 as a unit vector, and the two axes across it
        const int ex = part == 1, ey = part == 2, ez = part == 3;
        const int ux1 = !ex, uy1 = ex;  // y for the x axis, else x
        const int uy2 = ez, uz2 = !ez;  // y for the z axis, else z
        const int dn = up ? -1 : 1;     // change of the neighbours' up counts
        const uint32_t dc = dco_k;
        const DomainCoord c = {(int)(dc & 1023u), (int)((dc >> 10) & 1023u), (int)(dc >> 20)};
        const int endA = (int)(g.N / 8u);
        const __amdgpu_buffer_rsrc_t A =
            __builtin_amdgcn_make_buffer_rsrc((void *)g.A, (short)0, endA, 0x00020000);
        // gather: a neighbour across a face reads its spin and its other five
        // neighbours from memory (none of them flips in this cycle), both
        // neighbours' reads in flight together; one inside the octant reads LDS
        uint32_t wv[2][6];
        int bitp[2][6], cls[2], slab[2];
        bool across[2];
        uint32_t kj[2];
        int oj[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int side = e ? 1 : -1;
            const int x = lx + side * ex, y = ly + side * ey, z = lz + side * ez;
            const int along = ex ? x : ey ? y : z;
            across[e] = (unsigned)along > 15u;
            const int X = (so & 1) * 16 + x, Y = ((so >> 1) & 1) * 16 + y, Z = ((so >> 2) & 1) * 16 + z;
            const int PX[6] = {X, X + side * ex, X - ux1, X + ux1, X, X};
            const int PY[6] = {Y, Y + side * ey, Y - uy1, Y + uy1, Y - uy2, Y + uy2};
            const int PZ[6] = {Z, Z + side * ez, Z, Z, Z - uz2, Z + uz2};
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const int px = PX[i], py = PY[i], pz = PZ[i];
                const int cx = px < 0 ? wrapm(c.kx, g.nd) : px >= 32 ? wrapp(c.kx, g.nd) : c.kx;
                const int cy = py < 0 ? wrapm(c.ky, g.nd) : py >= 32 ? wrapp(c.ky, g.nd) : c.ky;
                const int cz = pz < 0 ? wrapm(c.kz, g.nd) : pz >= 32 ? wrapp(c.kz, g.nd) : c.kz;
                const int mx = px & 31, my = py & 31, mz = pz & 31;
                const int o = (mx >> 4) | ((my >> 4) << 1) | ((mz >> 4) << 2);
                const uint32_t kk = dindex(cx, cy, cz, g.nd);
                const uint32_t qq = (uint32_t)((mx & 15) + 16 * ((my & 15) + 16 * (mz & 15)));
                const int off = across[e] ? (int)(((kk * 8u + (uint32_t)o) * 128u + (qq >> 5)) * 4u) : endA;
                wv[e][i] = __builtin_amdgcn_raw_buffer_load_b32(A, off, 0, kCoherent);
                bitp[e][i] = (int)(qq & 31u);
                if (i == 0) {
                    kj[e] = kk;
                    oj[e] = o;
                    slab[e] = across[e] ? (mz & 15) >> 2 : z >> 2;
                }
            }
            // inside the octant: the class from LDS (a site inside stands in when across)
            cls[e] = slab_class_lds(o, across[e] ? lx : x, across[e] ? ly : y, across[e] ? lz : z);
        }
        // every read consumed before the first count move goes out
        int c_new[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t sj = (wv[e][0] >> bitp[e][0]) & 1u;
            int nup = (int)up;  // the flipped site, before its flip
#pragma unroll
            for (int i = 1; i < 6; ++i) nup += (int)((wv[e][i] >> bitp[e][i]) & 1u);
            const int up_j = cls[e] >= 7;
            const int nup_in = (up_j ? cls[e] - 7 : 6 - cls[e]);
            cls[e] = across[e] ? site_class(sj, nup) : cls[e];
            c_new[e] = across[e] ? site_class(sj, nup + dn) : site_class(up_j, nup_in + dn);
        }
        // (the classes pinned here: no count move may go out before both are known)
        asm volatile("" ::"v"(cls[0]), "v"(cls[1]), "v"(c_new[0]), "v"(c_new[1]) : "memory");
        // scatter: the class moves
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (across[e])
                slab_move_dev(g.sc + ((uint64_t)kj[e] * 8 + (uint32_t)oj[e]) * kSlabWords, cls[e],
                              c_new[e], slab[e]);
            else
                slab_move_lds(sc, cls[e], c_new[e], slab[e]);
        }
    }
}

// ALL: R_max over every octant of every domain (variant A): the counts of all
// eight octants are read every cycle, and every neighbour is waited for.
template <int BLOCK, bool ALL>
__device__ __forceinline__ void slab_body(const Replica &R, const uint32_t gid, SlabShared &sh) {
    static_assert(BLOCK == kSlabBlock, "one launch shape");
    const Geom &g = R.g;
    const PersistScratch &xs = R.xs;
    const uint64_t n0 = R.n0, ncycles = R.ncycles;
    const uint32_t obs_every = R.obs_every;
    constexpr int nthr = BLOCK, rows = kSlabRows, P = kSlabPasses;
    const int tid = threadIdx.x;
    const int row = tid >> 4, l = tid & 15;
    const uint32_t G = R.G;
    constexpr uint32_t D = kSlabDomains;
    const uint32_t kbase = gid * D;
    const uint32_t nvalid = kbase >= g.K ? 0u : (g.K - kbase < D ? g.K - kbase : D);
    const bool recorder = gid == 0;
    const uint64_t n_end = n0 + ncycles;

    for (uint32_t i = tid; i < 6 * (kMaxGrid / 32); i += nthr) (&sh.nbr_bits[0][0])[i] = 0;
    if (tid == 0) {
        sh.abort = 0;
        sh.pend_head = sh.pend_tail = 0;
    }
    load_predictions(sh, xs);
    if (tid < 14) sh.r[tid] = g.r[tid];
    if (l < 8) sh.zbuf[row][48 + l] = 0;
    for (uint32_t i = tid; i < nvalid * 6; i += nthr) {
        uint32_t ldm = i / 6;
        int dir = (int)(i % 6), a = dir >> 1;
        DomainCoord c = dcoord(kbase + ldm, g.nd);
        int kc[3] = {c.kx, c.ky, c.kz};
        kc[a] = (dir & 1) ? wrapp(kc[a], g.nd) : wrapm(kc[a], g.nd);
        sh.nbdom[ldm][dir] = dindex(kc[0], kc[1], kc[2], g.nd);
        if (dir == 0) sh.dco[ldm] = (uint32_t)c.kx | ((uint32_t)c.ky << 10) | ((uint32_t)c.kz << 20);
    }
    __syncthreads();
    for (uint32_t i = tid; i < nvalid * 6; i += nthr) {
        int dir = (int)(i % 6);
        uint32_t owner = sh.nbdom[i / 6][dir] / D;
        if (owner != gid) atomicOr(&sh.nbr_bits[dir][owner >> 5], 1u << (owner & 31));
    }
    __syncthreads();
    list_neighbours(sh, G);
    __syncthreads();

    // slab counts of all eight octants from the spins at launch start; they are
    // complete before this workgroup publishes its first R_max, hence before any
    // workgroup flips
#pragma unroll 1
    for (int o = 0; o < 8; ++o) slab_bin_octant(g, kbase, nvalid, o, sh);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    DevState *st = g.st;
    // launch-start totals: during a launch only the recorder writes them, at
    // its very end, after every workgroup has finished
    const uint64_t fired0 = st->fired, nulls0 = st->nulls;
    const int64_t M0 = st->M, B0 = st->B;
    double t = st->t;
    long long myF = 0, mydM = 0, mydB = 0;
    uint32_t rec_index = 0;
    int prev_colour = -1;
    double lnu = -log(cycle_draw(g.seed, n0, false).ut);
    uint64_t next_rec = obs_every ? (n0 / obs_every + 1) * obs_every : ~0ull;
    const int endSC = (int)((uint64_t)g.K * 8u * kSlabWords * 4u);
    const __amdgpu_buffer_rsrc_t SC = __builtin_amdgcn_make_buffer_rsrc((void *)g.sc, (short)0, endSC, 0x00020000);

    for (uint64_t n = n0; n < n_end; ++n) {
        const int s = cycle_draw(g.seed, n, false).colour;
        // the same colour again: the octants, halos and counts in LDS are current
        // (only this workgroup's own flips touched them, patched in below)
        const bool same = !ALL && n > n0 && s == prev_colour;
        // step 6 of the previous cycle: the flips (and count moves) that octant s can see
        if (ALL && n > n0) {
            if (!wait_neighbours<BLOCK>(xs, st, sh, G, -1, n)) break;
        } else if (n > n0) {
            int diff = s ^ prev_colour;
            if (diff && !(diff & (diff - 1))) {
                int a = diff == 1 ? 0 : diff == 2 ? 1 : 2;
                int dir = 2 * a + ((s >> a) & 1);
                if (!wait_neighbours<BLOCK>(xs, st, sh, G, dir, n)) break;
            }
        }
        prev_colour = s;

        // --- step 1 from the counts: the slab counts of the active octants first
        // (the frequency lines need only them), then their words and halos (only
        // the selection needs them: staged into LDS pass by pass just before it)
        // The counts go out with the first pass's words only; the other passes'
        // words follow once the counts are in, and arrive while the first
        // passes select.
        Raw<16> raw[P];
        if (!same) {
            // with ALL this cycle reads back the counts of the previous cycle's
            // octant, which this workgroup stored: those stores complete first
            if (ALL) __builtin_amdgcn_s_waitcnt(0);
            // lane c of a row: class c's slab counts (of every octant with ALL)
            constexpr int NO = ALL ? 8 : 1;
            uint32_t scw[P][NO][2];
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const bool valid = ld < nvalid;
#pragma unroll
                for (int oi = 0; oi < NO; ++oi) {
                    const uint32_t o = ALL ? (uint32_t)oi : (uint32_t)s;
                    const int off = valid && l < 14
                                        ? (int)((((kbase + ld) * 8u + o) * kSlabWords + 2u * (uint32_t)l) * 4u)
                                        : endSC;
                    const auto v = __builtin_amdgcn_raw_buffer_load_b64(SC, off, 0, kCoherent);
                    scw[pp][oi][0] = v[0];
                    scw[pp][oi][1] = v[1];
                }
            }
            load_octant<16>(g, kbase + (uint32_t)row, s, (uint32_t)row < nvalid, l,
                            sh.nbdom[(uint32_t)row < nvalid ? row : 0], raw[0]);
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                if (l < 14) {
#pragma unroll
                    for (int oi = 0; oi < NO; ++oi) {
                        const uint32_t w0 = scw[pp][oi][0], w1 = scw[pp][oi][1];
                        const int o = ALL ? oi : s;
                        sh.cnt[ld][o][l] = (uint16_t)((w0 & 0xFFFFu) + (w0 >> 16) + (w1 & 0xFFFFu) + (w1 >> 16));
                        if (o == s) {
                            sh.sc[ld][2 * l] = w0;
                            sh.sc[ld][2 * l + 1] = w1;
                        }
                    }
                }
            }
            // the previous cycle's count moves and stores are complete before this
            // workgroup's next R_max slot goes out (they are old by now)
            __builtin_amdgcn_s_waitcnt(0);
            asm volatile("" ::: "memory");  // the other passes' loads after the counts are in
#pragma unroll
            for (int pp = 1; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const bool valid = ld < nvalid;
                load_octant<16>(g, kbase + ld, s, valid, l, sh.nbdom[valid ? ld : 0], raw[pp]);
            }
        } else {
            __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                if (l < 14) {
                    const uint32_t v0 = sh.sc[ld][2 * l], v1 = sh.sc[ld][2 * l + 1];
                    sh.cnt[ld][s][l] = (uint16_t)((v0 & 0xFFFFu) + (v0 >> 16) + (v1 & 0xFFFFu) + (v1 >> 16));
                }
            }
        }
        if (ALL && tid < (int)D) sh.rk[tid] = 0.0;
        __syncthreads();
        if (ALL) {
            // every octant's frequency line; the active one keeps its running sums,
            // the domain's largest line goes into rk (non-negative doubles order as
            // their bit patterns)
            for (uint32_t i = tid; i < D * 8; i += nthr) {
                const uint32_t ld = i >> 3;
                const int o = (int)(i & 7u);
                double a = 0.0;
                for (int c = 0; c < 14; ++c) {
                    double term = (double)sh.cnt[ld][o][c] * sh.r[c];
                    a = a + term;
                    if (o == s) sh.acc[ld][c] = a;
                }
                if (ld < nvalid)
                    atomicMax(reinterpret_cast<unsigned long long *>(&sh.rk[ld]), (unsigned long long)double_to_bits(a));
            }
        } else {
            for (uint32_t i = tid; i < D; i += nthr) {
                double a = 0.0;
                for (int c = 0; c < 14; ++c) {
                    double term = (double)sh.cnt[i][s][c] * sh.r[c];
                    a = a + term;
                    sh.acc[i][c] = a;
                }
                sh.rk[i] = i < nvalid ? a : 0.0;
            }
        }
        __syncthreads();

        // --- step 2: R_max over all active octants (slot banks as in the re-binning engine)
        uint64_t *bank = xs.slot + (n & 1) * (uint64_t)G;
        const uint64_t gen = ((n >> 1) & 1) << 63;
        if (tid < 64) {
            double v = 0.0;
            for (uint32_t i = tid; i < D; i += 64) v = fmax(v, sh.rk[i]);
            v = wave_max_nonneg(v);
            if (tid == 63) st64(&bank[gid], double_to_bits(v) | gen);
        }
        // --- steps 3, 4 and 4b on the predicted R_max while the maxima travel
        U4 dw;
        {
            const uint32_t kd = kbase + (uint32_t)((l < P ? l : 0) * rows + row);
            dw = philox10((uint32_t)n, (uint32_t)(n >> 32), kd, (uint32_t)s, g.seed);
        }
        uint32_t cpred = 0;
        {
            const double Rspec = sh.rpred[s];
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                // this row's octant into LDS (the row's own lanes read it back)
                if (!same) {
                    uint32_t *o = sh.oct[ld];
#pragma unroll
                    for (int w = 0; w < 8; ++w) o[8 * l + w] = raw[pp].W[w];
                    // the six faces in the order of kFxm .. kFzp (one quarter-face per lane)
                    if (l < 12) *reinterpret_cast<uint4 *>(o + kFxm + 4 * l) = uint4{raw[pp].F[0], raw[pp].F[1], raw[pp].F[2], raw[pp].F[3]};
                }
                const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
                const int cs = row_class(sh.acc[ld], ld < nvalid, unit53(ux, uy) * Rspec, l, row);
                cpred |= (uint32_t)(cs + 1) << (5 * pp);
                slab_select(sh.sc[ld], sh.oct[ld], cs, uz, l, &sh.selq[ld], st);
            }
        }
        // the next cycle's draw (-ln u of its clock step, its colour), while the maxima travel
        const CycleDraw next_draw = cycle_draw(g.seed, n + 1, false);
        const double lnu_next = -log(next_draw.ut);
        // a neighbour reads this cycle's flips next cycle only if the next colour
        // differs from this one in one bit; otherwise they need only be complete
        // before the next R_max slot goes out (the wait before the next loads)
        const int next_diff = next_draw.colour ^ s;
        const bool last = n + 1 == n_end;
        const bool record = n + 1 == next_rec && g.rec_cap;
        const bool publish_flag = ALL || last || record || (next_diff && !(next_diff & (next_diff - 1)));
        if (tid < 64) {
            if (recorder && sh.pend_head != sh.pend_tail && sh.pend_cycle[sh.pend_head % kRecBanks] + 2 <= n + 1)
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
            uint64_t start = now_ticks();
            double best = 0.0;
            constexpr int kSlotsPerLane = 4;
            for (uint32_t base = 0; base < G && !sh.abort; base += 64 * kSlotsPerLane) {
                uint64_t sv[kSlotsPerLane];
#pragma unroll
                for (int i = 0; i < kSlotsPerLane; ++i) {
                    uint32_t w = base + (uint32_t)i * 64 + tid;
                    sv[i] = w < G ? ld64(&bank[w]) : gen;
                }
                for (;;) {
                    bool all = true;
#pragma unroll
                    for (int i = 0; i < kSlotsPerLane; ++i) {
                        uint32_t w = base + (uint32_t)i * 64 + tid;
                        if ((sv[i] & (1ull << 63)) != gen) {
                            all = false;
                            sv[i] = ld64(&bank[w]);
                        }
                    }
                    if (__all(all)) break;
                    __builtin_amdgcn_s_sleep(1);
                    if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                        atomicOr(&st->error, kErrBarrierTimeout);
                        sh.abort = 1;
                        break;
                    }
                }
#pragma unroll
                for (int i = 0; i < kSlotsPerLane; ++i) best = fmax(best, bits_to_double(sv[i] & ~(1ull << 63)));
            }
            best = wave_max_nonneg(best);
            if (tid == 63) sh.rmax = best;
        }
        __syncthreads();
        if (sh.abort) break;
        const double Rmax = sh.rmax;
        {
            if (tid == 0) sh.rpred[s] = Rmax;
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
                const int cs = row_class(sh.acc[ld], ld < nvalid, unit53(ux, uy) * Rmax, l, row);
                if ((uint32_t)(cs + 1) != ((cpred >> (5 * pp)) & 31u))
                    slab_select(sh.sc[ld], sh.oct[ld], cs, uz, l, &sh.selq[ld], st);
            }
        }
        __syncthreads();

        // --- the flips: four threads per domain, the flipped site (and its spin
        // word and halo copies) and its two neighbours along each axis.  A
        // neighbour inside the octant takes its class from the words in LDS (the
        // flipped site still reads its old spin there); one across a face reads
        // its own neighbours from memory (none of them flips in this cycle).
        {
            const uint32_t ld = (uint32_t)tid >> 2;
            const int part = tid & 3;
            const uint32_t f = ld < nvalid ? sh.selq[ld] : kNoEvent;
            if (f != kNoEvent)
                slab_flip_part(g, sh.oct[ld], sh.sc[ld], sh.dco[ld], sh.nbdom[ld], kbase + ld, s, f, part, myF, mydM,
                               mydB);
        }
        // this thread's flips and count moves complete (the flag below publishes them)
        if (publish_flag) __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // the flipped spins into the octants in LDS (read again if the colour repeats)
        if ((uint32_t)tid < nvalid && sh.selq[tid] != kNoEvent) {
            const uint32_t q = sh.selq[tid] & 0xFFFu;
            sh.oct[tid][q >> 5] ^= 1u << (q & 31);
        }
        // the active octants' counts back to memory (lane c of a row: class c).
        // Only this workgroup reads them, at the start of a later cycle, and no
        // other workgroup moves them before this workgroup's next R_max slot is
        // out: the wait for these stores sits before the next cycle's loads.
#pragma unroll
        for (int pp = 0; pp < P; ++pp) {
            const uint32_t ld = (uint32_t)(pp * rows + row);
            if (ld < nvalid && l < 14) {
                const uint64_t v = (uint64_t)sh.sc[ld][2 * l] | ((uint64_t)sh.sc[ld][2 * l + 1] << 32);
                st64(reinterpret_cast<uint64_t *>(g.sc + ((uint64_t)(kbase + ld) * 8 + (uint32_t)s) * kSlabWords +
                                                  2 * l),
                     v);
            }
        }
        // --- step 5: the clock
        {
            double dt = lnu / (8.0 * Rmax);
            t = t + dt;
        }
        lnu = lnu_next;
        __syncthreads();

        if (n + 1 == next_rec) next_rec += obs_every;
        if (record || last) {
            long long F = myF, dM = mydM, dB = mydB;
            for (int o = 32; o > 0; o >>= 1) {
                F += __shfl_xor(F, o);
                dM += __shfl_xor(dM, o);
                dB += __shfl_xor(dB, o);
            }
            if ((tid & 63) == 0) {
                sh.red[0][tid >> 6] = F;
                sh.red[1][tid >> 6] = dM;
                sh.red[2][tid >> 6] = dB;
            }
            __syncthreads();
            if (tid == 0) {
                F = dM = dB = 0;
                for (int w = 0; w < (nthr >> 6); ++w) {
                    F += sh.red[0][w];
                    dM += sh.red[1][w];
                    dB += sh.red[2][w];
                }
                if (last) {
                    // end of the launch: this workgroup's totals since launch start
                    store_final(xs, gid, F, dM, dB);
                } else {
                    const uint32_t bankr = rec_index % kRecBanks;
                    int64_t *rp = xs.recp + (uint64_t)bankr * G * 3;
                    st64((uint64_t *)&rp[3 * gid], (uint64_t)F);
                    st64((uint64_t *)&rp[3 * gid + 1], (uint64_t)dM);
                    st64((uint64_t *)&rp[3 * gid + 2], (uint64_t)dB);
                    if (recorder) {
                        const uint32_t slot = sh.pend_tail % kRecBanks;
                        sh.pend_cycle[slot] = n + 1;
                        sh.pend_t[slot] = t;
                        sh.pend_bank[slot] = bankr;
                        sh.pend_tail += 1;
                    }
                }
            }
            if (record && !last) rec_index += 1;
        }
        if (tid == 0 && publish_flag) {
            if (record || last) __builtin_amdgcn_s_waitcnt(0);
            st64(&xs.flag[gid], n + 1);
        }
    }

    // end of the launch: workgroup 0 waits for every workgroup, then appends the
    // pending records and the record of the last cycle
    if (recorder) {
        if (tid < 64 && !sh.abort) wait_all_flags(xs, st, sh, G, tid, n_end);
        __syncthreads();
        if (tid < 64 && !sh.abort) {
            while (sh.pend_head != sh.pend_tail) {
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
                __builtin_amdgcn_wave_barrier();
            }
            fold_final(g, xs, sh, G, tid, (uint64_t)g.K * ncycles, fired0, nulls0, M0, B0);
            if (tid == 0) {
                st->t = t;
                st->cycle = n_end;
                if (obs_every && (n_end % obs_every) == 0 && g.rec_cap) {
                    spkmc_record r;
                    r.cycle = n_end;
                    r.fired = st->fired;
                    r.nulls = st->nulls;
                    r.t = t;
                    r.M = st->M;
                    r.B = st->B;
                    g.rec[st->rec_count % g.rec_cap] = r;
                    st->rec_count += 1;
                }
            }
        }
    }
}

template <bool ALL>
__global__ void __launch_bounds__(kSlabBlock) k_slab(Replica R) {
    __shared__ SlabShared sh;
    slab_body<kSlabBlock, ALL>(R, blockIdx.x, sh);
}

// ---------------------------------------------------------------------------
// Per-cycle slab kernels (PACKED, octant edge 16, eight colours): one cycle in
// two launches from the slab counts, for lattices of any size.  k_srows_max
// takes every line's frequency line (every octant's with the all-octant R_max)
// from its count words and the largest into st->rmax[0]; k_srows_select stages
// each line's counts, octant and halo in LDS, draws, selects in one slab and
// flips (the class moves as in the slab engine).  The counts are binned once per
// run by k_slab_bin; kernel boundaries order every read after the writes it needs.
// ---------------------------------------------------------------------------
struct SrowsShared {
    alignas(16) uint32_t oct[kSlabDomains][kOctLds];
    uint32_t sc[kSlabDomains][kSlabWords];
    double acc[kSlabDomains][14];
    uint32_t nbdom[kSlabDomains][6];
    uint32_t dco[kSlabDomains];
    uint32_t selq[kSlabDomains];
    alignas(16) uint32_t zbuf[kSlabRows][kRowHalo];
    unsigned long long wmax;
    long long red[3][16];
};

// The slab counts of every octant of 128 domains per workgroup, from the spins.
__global__ void __launch_bounds__(kSlabBlock) k_slab_bin(Geom g) {
    __shared__ SrowsShared sh;
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
    const uint32_t kbase = blockIdx.x * kSlabDomains;
    const uint32_t nvalid = kbase >= g.K ? 0u : (g.K - kbase < kSlabDomains ? g.K - kbase : kSlabDomains);
    for (uint32_t i = tid; i < nvalid * 6; i += kSlabBlock) {
        const uint32_t ldm = i / 6;
        const int dir = (int)(i % 6), a = dir >> 1;
        const DomainCoord c = dcoord(kbase + ldm, g.nd);
        int kc[3] = {c.kx, c.ky, c.kz};
        kc[a] = (dir & 1) ? wrapp(kc[a], g.nd) : wrapm(kc[a], g.nd);
        sh.nbdom[ldm][dir] = dindex(kc[0], kc[1], kc[2], g.nd);
    }
    if (l < 8) sh.zbuf[row][48 + l] = 0;
    __syncthreads();
#pragma unroll 1
    for (int o = 0; o < 8; ++o) slab_bin_octant(g, kbase, nvalid, o, sh);
}

// Every line's frequency line from its count words (with the all-octant R_max:
// every octant of every domain), the largest into st->rmax[0].  One thread per
// line (or octant).
template <int LPD>
__global__ void __launch_bounds__(256) k_srows_max(Geom g, uint64_t n) {
    __shared__ unsigned long long wmax;
    const int tid = threadIdx.x;
    const bool all = (g.variant & SPKMC_VARIANT_RMAX_ALL) != 0;
    const uint32_t lpd = LPD ? (uint32_t)LPD : g.lpd;
    const uint64_t units = all ? (uint64_t)g.K * 8u : (uint64_t)g.K * lpd;
    const uint64_t u = (uint64_t)blockIdx.x * 256u + (uint64_t)tid;
    if (tid == 0) wmax = 0;
    __syncthreads();
    if (u < units) {
        const int s = cycle_draw(g.seed, n, lpd == 4).colour;
        uint32_t k, o;
        if (all) {
            k = (uint32_t)(u >> 3);
            o = (uint32_t)(u & 7u);
        } else {
            k = lpd == 1 ? (uint32_t)u : (uint32_t)(u >> 2);
            o = (uint32_t)(lpd == 1 ? s : two_colour_octant(s, (uint32_t)(u & 3u)));
        }
        const uint32_t *w = g.sc + ((uint64_t)k * 8u + o) * kSlabWords;
        uint32_t cnt[14];
#pragma unroll
        for (int c = 0; c < 14; ++c) {
            const uint32_t v0 = w[2 * c], v1 = w[2 * c + 1];
            cnt[c] = (v0 & 0xFFFFu) + (v0 >> 16) + (v1 & 0xFFFFu) + (v1 >> 16);
        }
        atomicMax(&wmax, (unsigned long long)double_to_bits(line_total(cnt, g.r)));
    }
    __syncthreads();
    if (tid == 0 && wmax) atomicMax((unsigned long long *)&g.st->rmax[0], wmax);
}

template <int LPD>
__global__ void __launch_bounds__(kSlabBlock) k_srows_select(Geom g, uint64_t n) {
    __shared__ SrowsShared sh;
    using RG = RowsGeometry<16, kSlabBlock, LPD, kSlabPasses>;
    constexpr int rows = RG::rows, P = RG::P;
    constexpr uint32_t D = RG::D;
    const RG rg(g);
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
    const int s = cycle_draw(g.seed, n, rg.lpd == 4).colour;
    const double Rmax = (g.variant & SPKMC_VARIANT_RMAX_BOUND) ? g.rbound : bits_to_double(g.st->rmax[0]);
    rg.neighbours(sh.nbdom);
    for (uint32_t i = tid; i < rg.nvalid; i += kSlabBlock) {
        const DomainCoord c = dcoord(rg.dom(rg.kbase + i), g.nd);
        sh.dco[i] = (uint32_t)c.kx | ((uint32_t)c.ky << 10) | ((uint32_t)c.kz << 20);
    }
    __syncthreads();
    // each line's counts (lane c: class c) and its octant and halo, into LDS
    const int endSC = (int)((uint64_t)g.K * 8u * kSlabWords * 4u);
    const __amdgpu_buffer_rsrc_t SC = __builtin_amdgcn_make_buffer_rsrc((void *)g.sc, (short)0, endSC, 0x00020000);
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < rg.nvalid;
        const uint32_t k = rg.dom(rg.kbase + ld), o = (uint32_t)rg.oct(rg.kbase + ld, s);
        const int off = valid && l < 14 ? (int)(((k * 8u + o) * kSlabWords + 2u * (uint32_t)l) * 4u) : endSC;
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(SC, off, 0, kCoherent);
        Raw<16> raw;
        load_octant<16>(g, k, (int)o, valid, l, sh.nbdom[valid ? ld : 0], raw);
        if (l < 14) {
            sh.sc[ld][2 * l] = v[0];
            sh.sc[ld][2 * l + 1] = v[1];
        }
        uint32_t *oc = sh.oct[ld];
#pragma unroll
        for (int w = 0; w < 8; ++w) oc[8 * l + w] = raw.W[w];
        if (l < 12) *reinterpret_cast<uint4 *>(oc + kFxm + 4 * l) = uint4{raw.F[0], raw.F[1], raw.F[2], raw.F[3]};
    }
    __syncthreads();
    // running sums of every line, in the order of step 1
    for (uint32_t i = tid; i < D; i += kSlabBlock) {
        double a = 0.0;
        for (int c = 0; c < 14; ++c) {
            const uint32_t v0 = sh.sc[i][2 * c], v1 = sh.sc[i][2 * c + 1];
            const uint32_t cnt = (v0 & 0xFFFFu) + (v0 >> 16) + (v1 & 0xFFFFu) + (v1 >> 16);
            double term = (double)cnt * g.r[c];
            a = a + term;
            sh.acc[i][c] = a;
        }
    }
    __syncthreads();
    // lane pp of each row draws for the row's line of pass pp
    U4 dw;
    {
        const uint32_t kd = rg.kbase + (uint32_t)((l < P ? l : 0) * rows + row);
        dw = philox10((uint32_t)n, (uint32_t)(n >> 32), rg.dom(kd), (uint32_t)rg.oct(kd, s), g.seed);
    }
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
        const int cs = row_class(sh.acc[ld], ld < rg.nvalid, unit53(ux, uy) * Rmax, l, row);
        slab_select(sh.sc[ld], sh.oct[ld], cs, uz, l, &sh.selq[ld], g.st);
    }
    __syncthreads();
    long long F = 0, dM = 0, dB = 0;
    {
        const uint32_t ld = (uint32_t)tid >> 2;
        const int part = tid & 3;
        const uint32_t f = ld < rg.nvalid ? sh.selq[ld] : kNoEvent;
        if (f != kNoEvent)
            slab_flip_part(g, sh.oct[ld], sh.sc[ld], sh.dco[ld], sh.nbdom[ld], rg.dom(rg.kbase + ld), rg.oct(rg.kbase + ld, s), f,
                           part, F, dM, dB);
    }
    __syncthreads();
    // the lines' counts back to memory (lane c of a row: class c)
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        if (ld < rg.nvalid && l < 14) {
            const uint32_t k = rg.dom(rg.kbase + ld), o = (uint32_t)rg.oct(rg.kbase + ld, s);
            *reinterpret_cast<uint64_t *>(g.sc + ((uint64_t)k * 8u + o) * kSlabWords + 2 * l) =
                (uint64_t)sh.sc[ld][2 * l] | ((uint64_t)sh.sc[ld][2 * l + 1] << 32);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        F += __shfl_xor(F, o);
        dM += __shfl_xor(dM, o);
        dB += __shfl_xor(dB, o);
    }
    if ((tid & 63) == 0) {
        sh.red[0][tid >> 6] = F;
        sh.red[1][tid >> 6] = dM;
        sh.red[2][tid >> 6] = dB;
    }
    __syncthreads();
    if (tid == 0) {
        F = dM = dB = 0;
        for (int w = 0; w < kSlabBlock / 64; ++w) {
            F += sh.red[0][w];
            dM += sh.red[1][w];
            dB += sh.red[2][w];
        }
        if (F) atomicAdd((unsigned long long *)&g.st->acc_fired[0], (unsigned long long)F);
        if (dM) atomicAdd((unsigned long long *)&g.st->acc_dM[0], (unsigned long long)dM);
        if (dB) atomicAdd((unsigned long long *)&g.st->acc_dB[0], (unsigned long long)dB);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Eight colours only: with two colours a neighbour across a face of a flipped
// site can have, diagonally, a site of another active octant that flips in the
// same cycle, and the two flips' class moves of that neighbour would each start
// from a stale class.  With eight colours that diagonal octant is never active.
bool slab_rows_supported(const Geom &g) {
    return g.layout == SPKMC_LAYOUT_PACKED && g.h == 16 && g.lpd == 1 && g.sc && g.N / 8 < (1ull << 31);
}

hipError_t launch_slab_bin(const Geom &g, hipStream_t stream) {
    if (!slab_rows_supported(g)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_slab_bin, dim3((g.K + kSlabDomains - 1) / kSlabDomains), dim3(kSlabBlock), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_cycle_slab(const Geom &g, uint64_t n, hipStream_t stream) {
    if (!slab_rows_supported(g)) return hipErrorInvalidValue;
    const uint64_t lines = (uint64_t)g.K * g.lpd;
    const uint32_t grid = (uint32_t)((lines + kSlabDomains - 1) / kSlabDomains);
    if (!(g.variant & SPKMC_VARIANT_RMAX_BOUND)) {
        const uint64_t units = (g.variant & SPKMC_VARIANT_RMAX_ALL) ? (uint64_t)g.K * 8u : lines;
        const uint32_t mgrid = (uint32_t)((units + 255) / 256);
        hipLaunchKernelGGL(k_srows_max<1>, dim3(mgrid), dim3(256), 0, stream, g, n);
    }
    hipLaunchKernelGGL(k_srows_select<1>, dim3(grid), dim3(kSlabBlock), 0, stream, g, n);
    return hipGetLastError();
}

static const void *slab_kernel(const Geom &g) {
    return (g.variant & SPKMC_VARIANT_RMAX_ALL) ? reinterpret_cast<const void *>(&k_slab<true>)
                                                : reinterpret_cast<const void *>(&k_slab<false>);
}

bool slab_supported(const Geom &g, const spkmc_params &p, std::string &why) {
    if (g.layout != SPKMC_LAYOUT_PACKED || g.h != 16) { why = "needs the PACKED layout and domain 32"; return false; }
    if (p.variant & ~(uint32_t)SPKMC_VARIANT_RMAX_ALL) { why = "runs variants 0 and RMAX_ALL"; return false; }
    if (g.N / 8 >= (1ull << 31)) { why = "needs fewer than 2^34 sites"; return false; }
    if (p.wg_domains && p.wg_domains != (int)kSlabDomains) { why = "takes 128 domains per workgroup"; return false; }
    return true;
}

hipError_t slab_configure(const Geom &g, int &grid, int &block, int &wg_domains) {
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, slab_kernel(g), kSlabBlock, 0);
    if (e != hipSuccess) return e;
    const uint64_t G = ((uint64_t)g.K + kSlabDomains - 1) / kSlabDomains;
    if (occ <= 0 || G > (uint64_t)occ * cus || G > (uint64_t)kMaxGrid) return hipErrorCooperativeLaunchTooLarge;
    grid = (int)G;
    block = kSlabBlock;
    wg_domains = (int)kSlabDomains;
    return hipSuccess;
}

hipError_t launch_slab(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid, bool prep,
                       hipStream_t stream) {
    if (!g.sc || g.h != 16) return hipErrorInvalidValue;
    PersistScratch xs = scratch_of(g, grid);
    if (prep) {
        hipError_t e = launch_persistent_prep(xs, (uint32_t)grid, n0, stream);
        if (e != hipSuccess) return e;
    }
    Replica R;
    R.g = g;
    R.xs = xs;
    R.n0 = n0;
    R.ncycles = ncycles;
    R.obs_every = obs_every;
    R.first_wg = 0;
    R.G = (uint32_t)grid;
    R.pad = 0;
    void *args[] = {&R};
    return hipLaunchCooperativeKernel(slab_kernel(g), dim3(grid), dim3(kSlabBlock), args, 0, stream);
}

}  // namespace spkmc
