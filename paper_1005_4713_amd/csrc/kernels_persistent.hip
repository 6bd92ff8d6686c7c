// kernels_persistent.hip -- the persistent ("PERSISTENT", "INCREMENTAL") engines
// of the gfx950 spkMC library: one cooperative launch runs many cycles (Sec. 3.1
// steps 1-6 with the sublattice steps 4a/4b of Sec. 3.2) over a bit-packed
// lattice; and the batch kernel (many lattices in one launch, also as a graph).
// The binning, selection and flip code is in persistent_common.hpp, shared with
// the per-cycle row kernels (kernels_rows.hip) and the slab engine
// (kernels_slab.hip).
//
// Work decomposition
//   * A 16-lane DPP row owns one frequency line (a domain's active octant); a
//     workgroup of B threads owns D = P * B / 16 consecutive lines (domains
//     numbered kx + nd (ky + nd kz)) for the whole launch, processed in P passes
//     whose class planes stay in registers from the bin to the flips.
//   * Each row selects on a predicted R_max (the last one of the same colour)
//     while the workgroup maxima travel, re-derives its class once the true
//     R_max is known and selects again only if the class changed; the event
//     goes into the row's selection slot in LDS, from which the flips are done.
//   * h = 16: lane l of the row holds plane lz = l of the octant (8 words, two
//     16-site x rows each); h = 8: lane l holds word l (four 8-site rows of
//     plane l / 2).  The z neighbours come from the adjacent lanes through DPP
//     row shifts, the y neighbours from the word below / above, the x
//     neighbours from in-word shifts; the 1-site halo comes from the face
//     copies of the six neighbouring octants (z faces staged per row in LDS).
//   * The up neighbours of 32 sites are counted bit-sliced (two full adders
//     and a 2-bit add, one v_bitop3 each), and the 14-class histogram of the
//     octant is recovered from 13 popcounts of products of the count bit planes
//     and the spin plane (inclusion-exclusion; n_up = 7 never occurs).
//
// Synchronisation (no cache-flushing fences: every word another workgroup may
// write is read with device-coherent loads, and every write is an atomic)
//   * R_max (step 2): each workgroup stores its local maximum into its own slot
//     of bank n & 1 with the generation (n >> 1) & 1 in the sign bit (all rates
//     are positive) and polls all slots of the bank; the maximum is exact and
//     order-free.  Two banks keep a fast workgroup's next value from
//     overwriting one a slow workgroup has not read yet.
//   * boundary events (step 6): after its flips a workgroup publishes the
//     cycle number in its flag.  Before binning cycle n + 1 a workgroup only
//     waits for the neighbouring workgroups the colour change s_n -> s_n+1
//     makes it depend on: the halo of colour s' holds flipped sites of colour
//     s_n only if s_n = s' ^ (1 << b), and then only from the neighbour domain
//     along axis b.  Flips of older cycles are covered by the R_max exchange
//     (a workgroup publishes its slot for cycle n only after its flips of
//     cycle n - 1 are complete).
//   * the clock (step 5) is advanced identically by every workgroup; each
//     workgroup stores its counter partials at an observation cycle, and
//     workgroup 0 sums them two cycles later while it waits for R_max.
// Every wait is bounded in wall-clock time; a timeout sets DevState::error and
// every workgroup leaves the loop.
#include <mutex>
#include <type_traits>
#include <string>

#include "persistent_common.hpp"

namespace spkmc {

// Workgroup-shared state of the persistent kernel for up to DMAX frequency lines
// (HISTP: with the incremental engine's packed counts of all eight octants; MW:
// moment words per line, 13 totals, or 36 for the one-round kernels' partial
// sums of four groups of four lanes, seven packed words and a spare each, and
// four words of padding: the histogram thread of line i reads line i's words as
// 16-byte loads, and a stride of 32 words would put the lanes of a wavefront on
// two bank offsets only).
template <uint32_t DMAX, bool HISTP, int MW>
struct PersistSharedT {
    double r[14];               // rate table
    alignas(16) uint32_t mom[DMAX][MW];  // per line: the popcount moments of its active octant
    uint32_t hist[DMAX][14];    // per line: class histogram (re-binning engine)
    uint32_t histp[HISTP ? DMAX : 1][8][7];  // per domain and octant: packed class counts (incremental engine)
    double acc[DMAX][14];       // per line: running FP64 sums of the frequency line
    double rk[DMAX];
    double uline[DMAX];         // per line: its event uniform of this cycle (speculative selection -> verification)
    alignas(16) uint32_t zbuf[64][kRowHalo];  // per row: the six halo faces (8 words each), zeros (8)
    uint32_t nbdom[DMAX][6];    // per line: its domain's neighbour domains -x, +x, -y, +y, -z, +z
    uint32_t selq[DMAX];        // per line: (class << 12) | site q of its event, or kNoEvent
    double rpred[8];                   // per colour: the last R_max seen (the prediction)
    double rmax;
    double next_lnu;                   // -ln u of the next cycle's clock step
    int next_colour;                   // the next cycle's colour
    int abort;
    uint32_t nbr_bits[6][kMaxGrid / 32];  // neighbour workgroups per direction, as a bitmap
    uint32_t nbr_cnt[6];                  // > kMaxNbr: too many, wait for every workgroup
    uint32_t nbr[6][kMaxNbr];
    long long red[3][16];
    // observation records whose partials are still to be summed (workgroup 0)
    uint32_t pend_head, pend_tail;
    uint64_t pend_cycle[kRecBanks];
    double pend_t[kRecBanks];
    uint32_t pend_bank[kRecBanks];
};
// The one-round re-binning kernels, and the incremental engine's (totals kept
// per line, and every octant's counts).
using PersistShared = PersistSharedT<kMaxWgDomains, false, 36>;
using PersistSharedInc = PersistSharedT<kMaxWgDomains, true, 13>;
// The wide mode (octant edge 16): RND = 2 or 4 rounds of four passes of 32 rows,
// 256 or 512 lines per workgroup.
template <int RND>
using PersistSharedWide = PersistSharedT<32 * 4 * RND, false, 13>;
static_assert(sizeof(PersistSharedWide<4>) <= 160 * 1024, "wide-mode LDS exceeds a CU's 160 KB");

// Bin octant o of every domain of the workgroup (the 13 moments of each row, then
// its histogram) into the packed counts of that octant.
template <int H, int P, int BLOCK>
__device__ __forceinline__ void bin_all(const Geom &g, uint32_t kbase, uint32_t nvalid, int o, PersistSharedInc &sh) {
    constexpr int rows = BLOCK / 16;
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
    constexpr uint32_t D = (uint32_t)(rows * P);
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < nvalid;
        Raw<H> raw;
        Planes<H> pl;
        load_octant<H>(g, kbase + ld, o, valid, l, sh.nbdom[valid ? ld : 0], raw);
        uint32_t m[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) m[i] = 0;
        compute_octant<H, true>(raw, valid, l, sh.zbuf[row], pl, m);
#pragma unroll
        for (int i = 0; i < 13; ++i) m[i] = row_scan(m[i]);
        if (l == 15) {
#pragma unroll
            for (int i = 0; i < 13; ++i) sh.mom[ld][i] = m[i];
        }
    }
    __syncthreads();
    for (uint32_t i = (uint32_t)tid; i < D; i += BLOCK) {
        uint32_t mm[13], hc[14];
        for (int c = 0; c < 13; ++c) mm[c] = sh.mom[i][c];
        hist_from_moments(mm, g.h3, hc);
        for (int c = 0; c < 14; c += 2) sh.histp[i][o][c >> 1] = i < nvalid ? (hc[c] | (hc[c + 1] << 16)) : 0u;
    }
    __syncthreads();
}

// INC = true: class histograms of all eight octants of every domain stay in LDS
// for the whole launch and follow every flip (the flipped site and its six
// neighbours change class, step 6); the active octant is classified only to
// find the selected site, while the R_max exchange is in flight.
// INC = false: the active octant of every domain is binned afresh each cycle.
// Lane j (0..15) of this thread's 16-lane row, for a j known only at run time.
__device__ __forceinline__ uint32_t row_lane(uint32_t v, int j) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(((threadIdx.x & 48u) + (uint32_t)j) << 2), (int)v);
}

// RND > 1 (the wide mode, re-binning engine only): each row runs RND rounds of P
// lines; the bin keeps only their moments, the selection waits for the true
// R_max and derives every round's class planes again from the spins.
// BND: 1 when the lattice may run with the fixed bound (read from the variant at
// run time), 0 when it does not (the bound's code is compiled out: present in the
// loop without running, it still slowed the cycle by about 2 %).
template <int H, int P, int BLOCK, bool INC, int LPD, int BND, int RND = 1,
          class SH = std::conditional_t<INC, PersistSharedInc, PersistShared>>
__device__ __forceinline__ void persistent_body(const Replica &R, const uint32_t gid, SH &sh) {
    static_assert(RND == 1 || (!INC && P * RND <= 16), "the wide mode re-bins; a row's lanes draw for its lines");
    static_assert(BLOCK >= 192, "the recorder sums records on its third wavefront");
    const Geom &g = R.g;
    const PersistScratch &xs = R.xs;
    const uint64_t n0 = R.n0, ncycles = R.ncycles;
    const uint32_t obs_every = R.obs_every;
    constexpr int nthr = BLOCK;
    constexpr int rows = BLOCK / 16;        // domains per pass
    const int tid = threadIdx.x;
    const int row = tid >> 4, l = tid & 15;  // DPP row and lane inside it
    const uint32_t G = R.G;
    const uint32_t D = (uint32_t)(rows * P * RND);
    // rows run frequency lines: one per domain, or (two colours) the four active
    // octants of each domain, lines 4k .. 4k + 3 of domain k
    const uint32_t lpd = LPD ? (uint32_t)LPD : g.lpd, NL = g.K * lpd;  // LPD = 0: read at run time
    const uint32_t kbase = gid * D;  // first line of the workgroup
    const uint32_t nvalid = kbase >= NL ? 0u : (NL - kbase < D ? NL - kbase : D);
    auto line_dom = [=](uint32_t line) { return lpd == 1 ? line : line >> 2; };
    auto line_oct = [=](uint32_t line, int colour) {
        return lpd == 1 ? colour : two_colour_octant(colour, line & 3u);
    };
    const bool recorder = gid == 0;
    const uint64_t n_end = n0 + ncycles;

    DevState *st = g.st;
    // launch-start totals: during a launch only the recorder writes them, at
    // its very end, after every workgroup has finished (read first, so that they
    // travel with the predictions' read below)
    const uint64_t fired0 = st->fired, nulls0 = st->nulls;
    const int64_t M0 = st->M, B0 = st->B;
    double t = st->t;  // every workgroup advances the same clock

    // neighbour workgroups per direction (0: -x, 1: +x, 2: -y, 3: +y, 4: -z, 5: +z)
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
        DomainCoord c = dcoord(line_dom(kbase + ldm), g.nd);
        int kc[3] = {c.kx, c.ky, c.kz};
        kc[a] = (dir & 1) ? wrapp(kc[a], g.nd) : wrapm(kc[a], g.nd);
        sh.nbdom[ldm][dir] = dindex(kc[0], kc[1], kc[2], g.nd);
    }
    __syncthreads();
    for (uint32_t i = tid; i < nvalid * 6; i += nthr) {
        int dir = (int)(i % 6);
        uint32_t owner = sh.nbdom[i / 6][dir] * lpd / D;
        if (owner != gid) atomicOr(&sh.nbr_bits[dir][owner >> 5], 1u << (owner & 31));
    }
    __syncthreads();
    list_neighbours(sh, G);
    __syncthreads();

    // INC: the histograms of all eight octants, from the spins at launch start
    // (no workgroup flips before every workgroup has published its first R_max)
    if constexpr (INC) {
#pragma unroll 1
        for (int o = 0; o < 8; ++o) bin_all<H, P, BLOCK>(g, kbase, nvalid, o, sh);
    }

    long long myF = 0, mydM = 0, mydB = 0;  // this thread's share since launch start
    uint32_t rec_index = 0;                  // records produced in this launch
    int prev_colour = -1;
    const bool bound = BND != 0 && (g.variant & SPKMC_VARIANT_RMAX_BOUND) != 0;  // re-binning engine only
    // the bound as a value: a conditional read of it or of an LDS word would be a
    // generic (flat) load, whose wait also waits for this wavefront's slot store
    const double rbound = g.rbound;
    const bool rmax_all = INC && (g.variant & SPKMC_VARIANT_RMAX_ALL);  // incremental engine only
    // the coming cycle's colour, and -ln u of its clock step (wavefront 0 keeps
    // the clock; the other wavefronts' t is never used)
    const CycleDraw cd0 = cycle_draw(g.seed, n0, lpd == 4);
    int s_next = cd0.colour;
    double lnu = 0.0;
    if (tid < 64) lnu = -log(cd0.ut);
    // the cycle after which the next observation record falls due
    uint64_t next_rec = obs_every ? (n0 / obs_every + 1) * obs_every : ~0ull;

    for (uint64_t n = n0; n < n_end; ++n) {
        const int s = s_next;  // the octant (eight colours) or the parity (two)

        // --- step 6 of the previous cycle: wait for the neighbour flips the halo of colour s can see.
        // With the fixed bound (no R_max exchange) or the all-octant maximum (every
        // octant's counts are needed) the wait covers every neighbour every cycle.
        if (n > n0) {
            if (bound || rmax_all) {
                if (!wait_neighbours<BLOCK>(xs, st, sh, G, -1, n)) break;
            } else if (lpd == 4) {
                // two colours: after a colour change every face of an active octant
                // touches the cells flipped in the previous cycle
                if (s != prev_colour && !wait_neighbours<BLOCK>(xs, st, sh, G, -1, n)) break;
            } else {
                int diff = s ^ prev_colour;
                if (diff && !(diff & (diff - 1))) {
                    int a = diff == 1 ? 0 : diff == 2 ? 1 : 2;
                    int dir = 2 * a + ((s >> a) & 1);  // below (-) if bit a of s is 0, else above (+)
                    if (!wait_neighbours<BLOCK>(xs, st, sh, G, dir, n)) break;
                }
            }
        }
        prev_colour = s;

        Planes<H> pl[P];
        // lane pp of each row draws for the row's line of pass pp; wavefronts with
        // no line to histogram draw while the others do (see below)
        U4 dw{};
        bool drawn = false;
        auto draw = [&]() {
            const uint32_t kd = kbase + (uint32_t)((l < P * RND ? l : 0) * rows + row);
            dw = philox10((uint32_t)n, (uint32_t)(n >> 32), line_dom(kd), (uint32_t)line_oct(kd, s), g.seed);
        };
        if constexpr (INC) {
            // --- fold the class changes other workgroups pushed into octant s (and,
            // every kFoldAll cycles, into all octants)
            const bool fold_all = rmax_all || (n - n0) % kFoldAll == kFoldAll - 1;
#pragma unroll 1
            for (int o = 0; o < 8; ++o) {
                if (o != s && !fold_all) continue;
                for (uint32_t i = tid; i < 2 * nvalid; i += nthr) {
                    uint64_t *w = g.dh + ((uint64_t)(kbase + (i >> 1)) * 8 + o) * 2 + (i & 1);
                    uint64_t v = ld64(w);
                    if (v) {
                        v = __hip_atomic_exchange(w, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (!fold_word(v, (int)(i & 1), sh.histp[i >> 1][o])) atomicOr(&st->error, kErrHist);
                    }
                }
            }
            __syncthreads();
            // --- step 1: frequency line of every domain from its counts (with the
            // all-octant maximum, rk is the largest line of the domain's octants)
            for (uint32_t i = tid; i < D; i += nthr) {
                const uint32_t *hp = sh.histp[i][s];
                double a = 0.0;
                for (int c = 0; c < 14; ++c) {
                    double term = (double)hcount(hp, c) * sh.r[c];
                    a = a + term;
                    sh.acc[i][c] = a;
                }
                double m = a;
                if (rmax_all) {
                    for (int o = 0; o < 8; ++o) {
                        const uint32_t *ho = sh.histp[i][o];
                        double b = 0.0;
                        for (int c = 0; c < 14; ++c) {
                            double term = (double)hcount(ho, c) * sh.r[c];
                            b = b + term;
                        }
                        m = fmax(m, b);
                    }
                }
                sh.rk[i] = i < nvalid ? m : 0.0;
            }
            __syncthreads();
        } else if constexpr (RND > 1) {
            // --- steps 1 and 4a, wide mode: the moments of every round's lines (the
            // class planes are derived again for the selection)
#pragma unroll 1
            for (int r = 0; r < RND; ++r) {
                Raw<H> raw[P];
#pragma unroll
                for (int pp = 0; pp < P; ++pp) {
                    const uint32_t ld = (uint32_t)((r * P + pp) * rows + row);
                    const bool valid = ld < nvalid;
                    load_octant<H>(g, line_dom(kbase + ld), line_oct(kbase + ld, s), valid, l,
                                   sh.nbdom[valid ? ld : 0], raw[pp]);
                }
#pragma unroll
                for (int pp = 0; pp < P; ++pp) {
                    const uint32_t ld = (uint32_t)((r * P + pp) * rows + row);
                    Planes<H> pw;
                    uint32_t m[13];
#pragma unroll
                    for (int i = 0; i < 13; ++i) m[i] = 0;
                    compute_octant<H, true>(raw[pp], ld < nvalid, l, sh.zbuf[row], pw, m);
                    uint32_t mp[7];
#pragma unroll
                    for (int i = 0; i < 6; ++i) mp[i] = row_scan(m[2 * i] | (m[2 * i + 1] << 16));
                    mp[6] = row_scan(m[12]);
                    if (l == 15) {
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            sh.mom[ld][2 * i] = mp[i] & 0xFFFFu;
                            sh.mom[ld][2 * i + 1] = mp[i] >> 16;
                        }
                        sh.mom[ld][12] = mp[6];
                    }
                }
            }
            __syncthreads();
            for (uint32_t i = tid; i < D; i += nthr) {
                uint32_t mm[13], hc[14];
                for (int c = 0; c < 13; ++c) mm[c] = sh.mom[i][c];
                hist_from_moments(mm, g.h3, hc);
                double a = 0.0;
                for (int c = 0; c < 14; ++c) {
                    double term = (double)hc[c] * sh.r[c];
                    a = a + term;
                    sh.acc[i][c] = a;
                    sh.hist[i][c] = hc[c];
                }
                sh.rk[i] = i < nvalid ? a : 0.0;
            }
            __syncthreads();
        } else {
            // --- steps 1 and 4a: class planes and moments of the active octants
            // (the words of every pass in flight at once; each pass's raw words
            // give way to its planes)
            Raw<H> raw[P];
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const bool valid = ld < nvalid;
                const uint32_t k = line_dom(kbase + ld);
                const int o = line_oct(kbase + ld, s);
                load_octant<H>(g, k, o, valid, l, sh.nbdom[valid ? ld : 0], raw[pp]);
            }
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                uint32_t ld = (uint32_t)(pp * rows + row);
                bool valid = ld < nvalid;
                uint32_t m[13];
#pragma unroll
                for (int i = 0; i < 13; ++i) m[i] = 0;
                compute_octant<H, true>(raw[pp], valid, l, sh.zbuf[row], pl[pp], m);
                // sums over groups of four lanes (two DPP steps; the last lane of a
                // group holds its group's), two moments to a word (at most h^3 <=
                // 4096 each); the histogram adds the four groups
                uint32_t mp[7];
#pragma unroll
                for (int i = 0; i < 6; ++i) mp[i] = quad_sum(m[2 * i] | (m[2 * i + 1] << 16));
                mp[6] = quad_sum(m[12]);
                if ((l & 3) == 3) {
                    uint32_t *dst = &sh.mom[ld][8 * (l >> 2)];
                    *reinterpret_cast<uint4 *>(dst) = uint4{mp[0], mp[1], mp[2], mp[3]};
                    *reinterpret_cast<uint4 *>(dst + 4) = uint4{mp[4], mp[5], mp[6], 0u};
                }
            }
            __syncthreads();
            if ((uint32_t)(tid & ~63) >= D) {  // no line of this wavefront to histogram
                draw();
                drawn = true;
            }
            // step 1: histogram and frequency line of every domain of the workgroup,
            // running sums kept for the selection (the same sums in the same order)
            for (uint32_t i = tid; i < D; i += nthr) {
                uint32_t mm[13], hc[14], w[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < 7; ++c) w[c] += sh.mom[i][8 * q + c];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    mm[2 * c] = w[c] & 0xFFFFu;
                    mm[2 * c + 1] = w[c] >> 16;
                }
                mm[12] = w[6];
                hist_from_moments(mm, g.h3, hc);
                double a = 0.0;
                for (int c = 0; c < 14; ++c) {
                    double term = (double)hc[c] * sh.r[c];
                    a = a + term;
                    sh.acc[i][c] = a;
                    sh.hist[i][c] = hc[c];
                }
                sh.rk[i] = i < nvalid ? a : 0.0;
            }
            __syncthreads();
        }

        // --- step 2: R_max over all active octants
        // bank n & 1 holds cycles n - 2 and n; the generation bit tells them apart
        uint64_t *bank = xs.slot + (n & 1) * (uint64_t)G;
        const uint64_t gen = ((n >> 1) & 1) << 63;
        if (tid < 64 && !bound) {
            double v = 0.0;
            for (uint32_t i = tid; i < D; i += 64) v = fmax(v, sh.rk[i]);
            v = wave_max_nonneg(v);
            if (tid == 63) st64(&bank[gid], double_to_bits(v) | gen);
        }
        if constexpr (INC) {
            // the active octants' class planes, while the other maxima travel
            Raw<H> raw[2];
            load_octant<H>(g, kbase + (uint32_t)row, s, (uint32_t)row < nvalid, l, sh.nbdom[row], raw[0]);
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                uint32_t ld = (uint32_t)(pp * rows + row);
                bool valid = ld < nvalid;
                if (pp + 1 < P) {
                    uint32_t ldn = ld + (uint32_t)rows;
                    load_octant<H>(g, kbase + ldn, s, ldn < nvalid, l, sh.nbdom[ldn < nvalid ? ldn : 0],
                                   raw[(pp + 1) & 1]);
                }
                uint32_t m[13];
                compute_octant<H, false>(raw[pp & 1], valid, l, sh.zbuf[row], pl[pp], m);
            }
        }
        // --- steps 3, 4 and 4b: event or null in every line.  The selection runs
        // first on a predicted R_max (the last one seen for this colour) while the
        // other workgroups' maxima travel; once the true R_max is known every row
        // re-derives its class with one ballot and selects again only if the class
        // changed, so the outcome is exactly that of the true R_max.
        if (!drawn) draw();
        // sites of class c on line ld
        auto line_count = [&](uint32_t ld, int c) -> uint32_t {
            return INC ? hcount(sh.histp[ld][s], c) : sh.hist[ld][c];
        };
        uint32_t cpred = 0;  // per pass: predicted class + 1, five bits each
        if constexpr (RND == 1) {
            const double Rspec = bound ? rbound : sh.rpred[s];
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
                const double u = unit53(ux, uy);
                if (l == 0) sh.uline[ld] = u;  // kept for the verification
                const int cs = row_class(sh.acc[ld], ld < nvalid, u * Rspec, l, row);
                cpred |= (uint32_t)(cs + 1) << (5 * pp);
                select_site<H>(pl[pp], cs, cs >= 0 ? line_count(ld, cs) : 0u, uz, l, &sh.selq[ld], st);
            }
        }

        // the next cycle's draw, by wavefront 1 while wavefront 0 polls
        if (tid == 64) {
            const CycleDraw nd = cycle_draw(g.seed, n + 1, lpd == 4);
            sh.next_colour = nd.colour;
            sh.next_lnu = -log(nd.ut);
        }

        // workgroup 0 sums a record stored two or more cycles ago on its third
        // wavefront, while the first polls
        if (recorder && !bound && (tid >> 6) == 2 && sh.pend_head != sh.pend_tail &&
            sh.pend_cycle[sh.pend_head % kRecBanks] + 2 <= n + 1)
            emit_record(g, xs, sh, G, tid & 63, n0, fired0, nulls0, M0, B0);
        if (tid < 64 && !bound) {
            // poll every slot until all carry this cycle's generation: one round of
            // loads for a block of slots, then only the ones not yet there
            uint64_t start = now_ticks();
            double best = 0.0;
            constexpr int kSlotsPerLane = 4;  // 256 slots per round of the first wave
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
        const double Rmax = bound ? rbound : sh.rmax;
        s_next = sh.next_colour;

        if constexpr (RND > 1) {
            // --- steps 3, 4 and 4b, wide mode: every round's class planes from its
            // words, then the selection with the true R_max
#pragma unroll 1
            for (int r = 0; r < RND; ++r) {
                Raw<H> raw[P];
#pragma unroll
                for (int pp = 0; pp < P; ++pp) {
                    const uint32_t ld = (uint32_t)((r * P + pp) * rows + row);
                    const bool valid = ld < nvalid;
                    load_octant<H>(g, line_dom(kbase + ld), line_oct(kbase + ld, s), valid, l,
                                   sh.nbdom[valid ? ld : 0], raw[pp]);
                }
#pragma unroll
                for (int pp = 0; pp < P; ++pp) {
                    const int j = r * P + pp;
                    const uint32_t ld = (uint32_t)(j * rows + row);
                    const bool valid = ld < nvalid;
                    Planes<H> pw;
                    uint32_t m[13];
                    compute_octant<H, false>(raw[pp], valid, l, sh.zbuf[row], pw, m);
                    const uint32_t ux = row_lane(dw.x, j), uy = row_lane(dw.y, j), uz = row_lane(dw.z, j);
                    const int cs = row_class(sh.acc[ld], valid, unit53(ux, uy) * Rmax, l, row);
                    select_site<H>(pw, cs, cs >= 0 ? sh.hist[ld][cs] : 0u, uz, l, &sh.selq[ld], st);
                }
            }
        } else if (!bound) {
            // the true R_max: rows whose class differs select again
            if (tid == 0) sh.rpred[s] = Rmax;
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const int cs = row_class(sh.acc[ld], ld < nvalid, sh.uline[ld] * Rmax, l, row);
                if ((uint32_t)(cs + 1) != ((cpred >> (5 * pp)) & 31u))
                    select_site<H>(pl[pp], cs, cs >= 0 ? line_count(ld, cs) : 0u, bcast_lane(dw.z, pp), l,
                                   &sh.selq[ld], st);
            }
        }
        __syncthreads();
        // --- the flips of this cycle
        // one thread per row with an event; incremental engine: three threads per
        // such row, one per axis, each moving the
        // classes of the flipped site's two neighbours along its axis; the first
        // also flips the site (spin word and halo copies) and moves its class
        const uint32_t nwork = INC ? 3 * D : D;
        for (uint32_t t = tid; t < nwork; t += nthr) {
            const uint32_t ld = INC ? t / 3 : t, ax = INC ? t % 3 : 0;
            const uint32_t f = sh.selq[ld];
            if (f == kNoEvent) continue;
            const uint32_t cs = f >> 12, q = f & 0xFFFu;
            const uint32_t k = line_dom(kbase + ld);
            const int so = line_oct(kbase + ld, s);  // the line's octant
            if constexpr (INC) {
                // The neighbours' other neighbours do not change in this cycle (one flip
                // per domain, and same-coloured octants of different domains never
                // touch), so their classes follow from spins read now, with the flipped
                // site's spin taken before its flip.  The twelve reads are independent.
                const int qc[3] = {(int)(q % H), (int)((q / H) % H), (int)(q / (H * H))};
                const int Q[3] = {(so & 1) * H + qc[0], ((so >> 1) & 1) * H + qc[1], ((so >> 2) & 1) * H + qc[2]};
                const uint32_t up = cs >= 7;
                const int dn = up ? -1 : 1;  // change of the neighbours' up counts
                const DomainCoord dc = dcoord(k, g.nd);
                const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;  // the other two axes
                uint32_t sj[2], kj[2];
                int oj[2], nup[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int side = e ? 1 : -1;
                    int J[3] = {Q[0], Q[1], Q[2]};
                    J[ax] += side;
                    uint32_t kt;
                    int ot;
                    sj[e] = spin_at<H>(g, dc, J, kj[e], oj[e]);
                    nup[e] = (int)up;
                    int T[3] = {J[0], J[1], J[2]};
                    T[ax] += side;
                    nup[e] += (int)spin_at<H>(g, dc, T, kt, ot);
                    T[ax] = J[ax];
                    T[b1] -= 1;
                    nup[e] += (int)spin_at<H>(g, dc, T, kt, ot);
                    T[b1] += 2;
                    nup[e] += (int)spin_at<H>(g, dc, T, kt, ot);
                    T[b1] = J[b1];
                    T[b2] -= 1;
                    nup[e] += (int)spin_at<H>(g, dc, T, kt, ot);
                    T[b2] += 2;
                    nup[e] += (int)spin_at<H>(g, dc, T, kt, ot);
                }
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int c_old = site_class(sj[e], nup[e]), c_new = site_class(sj[e], nup[e] + dn);
                    if (kj[e] - kbase < nvalid) {
                        hmove(sh.histp[kj[e] - kbase][oj[e]], c_old, c_new);
                    } else {
                        (void)__hip_atomic_fetch_add(g.dh + ((uint64_t)kj[e] * 8 + oj[e]) * 2 + sj[e],
                                                     digit_move(c_old - 7 * (int)sj[e], c_new - 7 * (int)sj[e]),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                if (ax != 0) continue;
                hmove(sh.histp[ld][so], cs, site_class(!up, up ? cs - 7 : 6 - cs));
            }
            flip_site<H>(g, k, so, q, sh.nbdom[ld]);
            myF += 1;
            mydM += cs >= 7 ? -2 : 2;              // the class carries the old spin
            mydB += 12 - 4 * (long long)(cs % 7);  // and its aligned count
        }

        // this thread's flips complete (its only memory operations in flight) when
        // the next cycle reads what they changed: the same colour again (this
        // workgroup reloads its octants) or a colour one bit away (neighbours wait for
        // the flag).  Otherwise the next cycle's loads, issued after them, wait for
        // them, which its R_max publish follows.
        const int dn_next = s ^ s_next;
        const bool indep = !INC && RND == 1 && !bound && lpd == 1 && n + 1 < n_end && (dn_next & (dn_next - 1)) != 0;
        if (!indep) __builtin_amdgcn_s_waitcnt(0);

        // --- step 5: the clock, identical in every workgroup
        if (tid < 64) {
            double dt = lnu / ((lpd == 4 ? 2.0 : 8.0) * Rmax);
            t = t + dt;
            lnu = sh.next_lnu;
        }
        // flips complete, then publish them (step 6)
        __syncthreads();

        const bool last = n + 1 == n_end;
        const bool record = n + 1 == next_rec && g.rec_cap;
        if (n + 1 == next_rec) next_rec += obs_every;
        if (record || last) {
            // workgroup totals since launch start
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
                    const uint32_t bank = rec_index % kRecBanks;
                    if (bound) {
                        // no R_max exchange keeps the workgroups within a cycle of one
                        // another: before reusing a bank wait until workgroup 0 has
                        // appended the record that used it
                        const uint64_t start = now_ticks();
                        while (ld64(xs.emitted) + kRecBanks <= rec_index) {
                            __builtin_amdgcn_s_sleep(1);
                            if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                                atomicOr(&st->error, kErrFlagTimeout);
                                sh.abort = 1;
                                break;
                            }
                        }
                    }
                    int64_t *rp = xs.recp + (uint64_t)bank * G * 3;
                    st64((uint64_t *)&rp[3 * gid], (uint64_t)F);
                    st64((uint64_t *)&rp[3 * gid + 1], (uint64_t)dM);
                    st64((uint64_t *)&rp[3 * gid + 2], (uint64_t)dB);
                    if (recorder) {
                        const uint32_t slot = sh.pend_tail % kRecBanks;
                        sh.pend_cycle[slot] = n + 1;
                        sh.pend_t[slot] = t;
                        sh.pend_bank[slot] = bank;
                        sh.pend_tail += 1;
                    }
                }
            }
            if (record && !last) rec_index += 1;
        }
        if (tid == 0) {
            // the record partials stored above go out first; the flips are complete
            // (each thread waited for its own before the barrier)
            if (!indep) {
                if (record || last) __builtin_amdgcn_s_waitcnt(0);
                st64(&xs.flag[gid], n + 1);
            }
        }
        if (bound && record && !last) {  // uniform over the workgroup
            if (recorder && tid < 64) {
                // fixed bound: workgroup 0 appends the record as soon as every
                // workgroup has completed the cycle (its own flag is already out)
                if (wait_all_flags(xs, st, sh, G, tid, n + 1)) {
                    emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
                    if (tid == 0) st64(xs.emitted, (uint64_t)rec_index);
                }
            }
            __syncthreads();
            if (sh.abort) break;
        }
    }

    // end of the launch: workgroup 0 waits for every workgroup to finish, then
    // appends the records still pending and the record of the last cycle
    if (recorder) {
        if (tid < 64 && !sh.abort) wait_all_flags(xs, st, sh, G, tid, n_end);
        __syncthreads();
        if (tid < 64 && !sh.abort) {
            while (sh.pend_head != sh.pend_tail) {
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
                __builtin_amdgcn_wave_barrier();
            }
            fold_final(g, xs, sh, G, tid, NL * ncycles, fired0, nulls0, M0, B0);
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

// One lattice: the descriptor by value; LPD, the frequency lines per domain (1
// or 4), fixed at compile time so that every line of a pass shares its octant.
template <int H, int P, int BLOCK, bool INC, int LPD, int BND>
__global__ void __launch_bounds__(BLOCK) k_persistent(Replica R) {
    __shared__ std::conditional_t<INC, PersistSharedInc, PersistShared> sh;
    persistent_body<H, P, BLOCK, INC, LPD, BND>(R, blockIdx.x, sh);
}

// One lattice in the wide mode (octant edge 16; RND rounds of four passes, 128 RND
// lines per workgroup).
template <int RND, int LPD, int BND>
__global__ void __launch_bounds__(512) k_persistent_wide(Replica R) {
    __shared__ PersistSharedWide<RND> sh;
    persistent_body<16, 4, 512, false, LPD, BND, RND, PersistSharedWide<RND>>(R, blockIdx.x, sh);
}

// Many independent lattices in one launch: each workgroup finds its lattice by
// its workgroup index; lattices never wait for one another.
// LPD: 1 when every lattice of the batch has eight colours (one line per domain,
// fixed at compile time) and none the fixed bound; 0 for batches that mix in
// two-colour or fixed-bound lattices (both read at run time).
template <int H, int P, int BLOCK, bool INC, int LPD>
__global__ void __launch_bounds__(BLOCK) k_persistent_batch(const Replica *__restrict__ reps, uint32_t nrep) {
    __shared__ PersistShared sh;
    uint32_t lo = 0, hi = nrep;  // last replica with first_wg <= blockIdx.x
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (reps[mid].first_wg <= blockIdx.x) lo = mid;
        else hi = mid;
    }
    // the index is the same in every lane: keep the descriptor in scalar registers
    const Replica &R = reps[__builtin_amdgcn_readfirstlane(lo)];
    if (blockIdx.x >= R.first_wg + R.G) return;  // a spare workgroup past the last lattice
    persistent_body<H, P, BLOCK, INC, LPD, LPD == 0 ? 1 : 0>(R, blockIdx.x - R.first_wg, sh);
}

// Before a launch: slots carry the generation of no cycle of this launch yet,
// flags the start cycle.  (The end of a launch of at least two cycles leaves
// both in exactly this state for a launch of the same shape that continues
// where it stopped.)
__device__ __forceinline__ void prep_one(const PersistScratch &xs, uint32_t G, uint64_t n0, uint32_t i) {
    // bank b first serves cycle nb (n0 or n0 + 1, nb & 1 == b): mark it "not yet"
    for (uint64_t nb = n0; nb < n0 + 2; ++nb) xs.slot[(nb & 1) * G + i] = (((nb >> 1) + 1) & 1) << 63;
    xs.flag[i] = n0;
    if (i == 0) *xs.emitted = 0;
}
// and (incremental engine) no pushed class changes pending: the launch starts
// from histograms binned afresh.
__global__ void k_persistent_prep(PersistScratch xs, uint32_t G, uint64_t n0, uint64_t *dh, uint64_t ndh) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G) prep_one(xs, G, n0, (uint32_t)i);
    for (uint64_t w = i; w < ndh; w += (uint64_t)gridDim.x * blockDim.x) dh[w] = 0;
}
__global__ void k_persistent_prep_batch(const Replica *__restrict__ reps, uint32_t nrep, int zero_dh) {
    for (uint32_t r = blockIdx.x; r < nrep; r += gridDim.x) {
        for (uint32_t i = threadIdx.x; i < reps[r].G; i += blockDim.x) prep_one(reps[r].xs, reps[r].G, reps[r].n0, i);
        if (zero_dh) {
            const uint64_t ndh = (uint64_t)reps[r].g.K * 16;
            for (uint64_t w = threadIdx.x; w < ndh; w += blockDim.x) reps[r].g.dh[w] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Launch shapes.  A 16-lane row owns a domain; a workgroup runs `rows` rows
// and P passes (1, 2 or 4).  h = 16 keeps up to four passes of class planes in
// 256 registers with 32 rows (512 threads, two waves per SIMD); h = 8 needs 4
// registers per pass and runs 64 rows (1024 threads, four waves per SIMD).
// The incremental engine keeps more state per line than re-binning (counts of
// all eight octants, pushed changes): 32 rows and at most two passes, so that
// its kernels fit their registers.
int persist_rows(int h, bool inc) { return h == 8 && !inc ? 64 : 32; }
int persist_max_passes(int, bool inc) { return inc ? 2 : 4; }
// Batches of octant edge 8 (1024 threads, 128 registers) stop at two passes:
// with four the batch kernel's run-time descriptor spills registers.
int batch_max_passes(int h) { return h == 8 ? 2 : 4; }

// batch: lpd = 1 (every lattice with eight colours and without the fixed bound)
// or 0 (lines per domain and the bound read at run time).  Single lattices: bnd,
// the lattice runs with the fixed bound.
template <int H, int P, int BLOCK>
static void *kernel_of(bool batch, bool inc, uint32_t lpd, bool bnd) {
    if (inc) {
        if constexpr (P <= 2 && BLOCK == 512) return reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, true, 1, 0>);
        return nullptr;
    }
    if (batch)
        return lpd == 1 ? reinterpret_cast<void *>(&k_persistent_batch<H, P, BLOCK, false, 1>)
                        : reinterpret_cast<void *>(&k_persistent_batch<H, P, BLOCK, false, 0>);
    if (bnd)
        return lpd == 4 ? reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 4, 1>)
                        : reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 1, 1>);
    return lpd == 4 ? reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 4, 0>)
                    : reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 1, 0>);
}

// The wide mode's rounds for one lattice: 1 (passes only), 2 or 4 (octant edge 16,
// re-binning engine).
static int max_rounds(int h, bool inc) { return h == 16 && !inc ? 4 : 1; }

static bool has_bound(const Geom &g) { return (g.variant & SPKMC_VARIANT_RMAX_BOUND) != 0; }

template <int RND>
static void *wide_kernel(uint32_t lpd, bool bnd) {
    if (bnd)
        return lpd == 4 ? reinterpret_cast<void *>(&k_persistent_wide<RND, 4, 1>)
                        : reinterpret_cast<void *>(&k_persistent_wide<RND, 1, 1>);
    return lpd == 4 ? reinterpret_cast<void *>(&k_persistent_wide<RND, 4, 0>)
                    : reinterpret_cast<void *>(&k_persistent_wide<RND, 1, 0>);
}

// Batches use the re-binning kernel (see kernel_of for lpd and bnd).
static void *select_kernel(int h, int P, int block, bool batch = false, bool inc = false, uint32_t lpd = 1,
                           int rnd = 1, bool bnd = false) {
    if (batch && inc) return nullptr;
    if (rnd > 1) {
        if (batch || inc || h != 16 || block != 512 || P != 4) return nullptr;
        if (rnd == 2) return wide_kernel<2>(lpd, bnd);
        if (rnd == 4) return wide_kernel<4>(lpd, bnd);
        return nullptr;
    }
    if (h == 16 && block == 512)
        return P == 1   ? kernel_of<16, 1, 512>(batch, inc, lpd, bnd)
               : P == 2 ? kernel_of<16, 2, 512>(batch, inc, lpd, bnd)
               : P == 4 ? kernel_of<16, 4, 512>(batch, inc, lpd, bnd)
                        : nullptr;
    if (h == 8 && block == 1024 && !inc)
        return P == 1   ? kernel_of<8, 1, 1024>(batch, inc, lpd, bnd)
               : P == 2 ? kernel_of<8, 2, 1024>(batch, inc, lpd, bnd)
               : P == 4 ? kernel_of<8, 4, 1024>(batch, inc, lpd, bnd)
                        : nullptr;
    if (h == 8 && block == 512 && inc && !batch)
        return P == 1   ? kernel_of<8, 1, 512>(false, true, 1, false)
               : P == 2 ? kernel_of<8, 2, 512>(false, true, 1, false)
                        : nullptr;
    return nullptr;
}

bool persistent_supported(const Geom &g, const spkmc_params &p, bool inc, std::string &why) {
    if (g.layout != SPKMC_LAYOUT_PACKED) { why = "needs the PACKED layout"; return false; }
    if (g.h != 8 && g.h != 16) { why = "needs an octant edge of 8 or 16 (domain 16 or 32)"; return false; }
    // spins and halo copies are read through buffer views with 32-bit byte offsets
    if (g.N / 8 >= (1ull << 31)) { why = "needs fewer than 2^34 sites"; return false; }
    const uint32_t ok = inc ? SPKMC_VARIANT_RMAX_ALL : (SPKMC_VARIANT_RMAX_BOUND | SPKMC_VARIANT_TWO_COLOURS);
    if (p.variant & ~ok) {
        why = inc ? "the incremental engine runs variants 0 and RMAX_ALL"
                  : "this engine runs variants 0, RMAX_BOUND and TWO_COLOURS";
        return false;
    }
    const int rows = persist_rows(g.h, inc), pmax = persist_max_passes(g.h, inc) * max_rounds(g.h, inc);
    const int pc = p.wg_domains / rows;
    if (p.wg_domains && (p.wg_domains % rows || pc > pmax || (pc & (pc - 1)))) {
        why = "wg_domains must be " + std::to_string(rows) + " times a power of two up to " + std::to_string(pmax) +
              " for this octant edge and engine";
        return false;
    }
    return true;
}

hipError_t persistent_configure(const Geom &g, const spkmc_params &p, bool inc, int &grid, int &block,
                                int &wg_domains) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int rows = persist_rows(g.h, inc), pmax = persist_max_passes(g.h, inc);
    block = rows * 16;
    // the fewest passes (then rounds of passes) whose workgroups are all resident
    // at once (or the requested lines per workgroup)
    for (int pc = 1; pc <= pmax * max_rounds(g.h, inc); pc <<= 1) {
        const int P = pc < pmax ? pc : pmax;
        if (p.wg_domains && p.wg_domains != rows * pc) continue;
        void *kern = select_kernel(g.h, P, block, false, inc, g.lpd, pc / P, has_bound(g));
        if (!kern) return hipErrorInvalidValue;
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, 0);
        if (e != hipSuccess) return e;
        const uint64_t D = (uint64_t)rows * pc, G = ((uint64_t)g.K * g.lpd + D - 1) / D;
        if (occ > 0 && G <= (uint64_t)occ * cus && G <= (uint64_t)kMaxGrid) {
            grid = (int)G;
            wg_domains = (int)D;
            return hipSuccess;
        }
    }
    return hipErrorCooperativeLaunchTooLarge;
}

uint64_t persistent_scratch_words(uint64_t K) { return kScratchWordsPerWg * (K / 16 + 2) + 16; }

PersistScratch scratch_of(const Geom &g, int G) {
    PersistScratch xs;
    xs.slot = g.sync;
    xs.flag = g.sync + 2 * (uint64_t)G;
    xs.recp = reinterpret_cast<int64_t *>(g.sync + 3 * (uint64_t)G);
    xs.fin = reinterpret_cast<int64_t *>(g.sync + 15 * (uint64_t)G);
    xs.emitted = g.sync + 18 * (uint64_t)G;                  // within the 16 spare words
    xs.rpred = reinterpret_cast<double *>(xs.emitted + 1);  // 8 more of them
    return xs;
}

hipError_t launch_persistent(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid, int block,
                             int wg_domains, bool inc, bool prep, hipStream_t stream) {
    PersistScratch xs = scratch_of(g, grid);
    const int pc = wg_domains / (block / 16), P = pc < 4 ? pc : 4;  // passes, then rounds of four passes
    void *kern = select_kernel(g.h, P, block, false, inc, g.lpd, pc / P, has_bound(g));
    if (!kern) return hipErrorInvalidValue;
    if (prep || inc) {  // the incremental engine clears its pushed class changes every launch
        const uint64_t ndh = inc ? (uint64_t)g.K * 16 : 0;
        uint64_t blocks = ((uint64_t)grid + 255) / 256, bdh = (ndh + 255) / 256;
        blocks = blocks > bdh ? blocks : (bdh < 2048 ? bdh : 2048);
        hipLaunchKernelGGL(k_persistent_prep, dim3((uint32_t)blocks), dim3(256), 0, stream, xs, (uint32_t)grid, n0,
                           g.dh, ndh);
        hipError_t e = hipGetLastError();
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
    return hipLaunchCooperativeKernel(kern, dim3(grid), dim3(block), args, 0, stream);
}

hipError_t launch_persistent_prep(const PersistScratch &xs, uint32_t G, uint64_t n0, hipStream_t stream) {
    hipLaunchKernelGGL(k_persistent_prep, dim3((G + 255) / 256), dim3(256), 0, stream, xs, G, n0, (uint64_t *)nullptr,
                       (uint64_t)0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batches: one cooperative launch over several lattices of the same octant edge
// ---------------------------------------------------------------------------
size_t replica_bytes() { return sizeof(Replica); }

// Workgroups lattice i needs with `rows_pp` domains per pass and P passes.
uint32_t batch_wgs(const Geom &g, int P) {
    const uint64_t D = (uint64_t)persist_rows(g.h, false) * P;
    return (uint32_t)(((uint64_t)g.K * g.lpd + D - 1) / D);
}

// Workgroups of the batch kernel for octant edge h and P passes that the
// current device keeps resident at once (0 on error).
uint32_t batch_capacity(int h, int P, uint32_t lpd) {
    const int block = persist_rows(h, false) * 16;
    void *kern = select_kernel(h, P, block, true, false, lpd);
    if (!kern) return 0;
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, 0) != hipSuccess) return 0;
    uint64_t cap = (uint64_t)occ * (uint64_t)cus;
    return (uint32_t)(cap < kMaxGrid ? cap : kMaxGrid);
}

// Fill the descriptors (host memory) and check the launch fits on the device.
hipError_t batch_plan(const Geom *const *gs, const uint64_t *n0, const uint64_t *ncycles, uint32_t obs_every,
                      uint32_t n, int P, Replica *out, int &grid, int &block, uint32_t &lpd) {
    if (n == 0) return hipErrorInvalidValue;
    const int h = gs[0]->h;
    block = persist_rows(h, false) * 16;
    lpd = 1;
    for (uint32_t i = 0; i < n; ++i)
        if (gs[i]->lpd != 1 || has_bound(*gs[i])) lpd = 0;
    void *kern = select_kernel(h, P, block, true, false, lpd);
    if (!kern) return hipErrorInvalidValue;
    uint32_t first = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (gs[i]->h != h) return hipErrorInvalidValue;
        out[i].g = *gs[i];
        out[i].G = batch_wgs(*gs[i], P);
        out[i].xs = scratch_of(*gs[i], (int)out[i].G);
        out[i].n0 = n0[i];
        out[i].ncycles = ncycles[i];
        out[i].obs_every = obs_every;
        out[i].first_wg = first;
        out[i].pad = 0;
        first += out[i].G;
    }
    const uint32_t cap = batch_capacity(h, P, lpd);
    if (cap == 0) return hipErrorInvalidValue;
    if (first > cap) return hipErrorCooperativeLaunchTooLarge;
    grid = (int)first;
    return hipSuccess;
}

// Descriptors reach device memory as kernel arguments (copied at launch, so the
// host array may go away at once): up to kUploadPer per launch.
constexpr uint32_t kUploadPer = 8;
struct ReplicaPack {
    Replica r[kUploadPer];
};
__global__ void k_upload(ReplicaPack pack, uint32_t count, Replica *dst) {
    const uint32_t words = (uint32_t)(sizeof(Replica) / sizeof(uint32_t));
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&pack);
    uint32_t *out = reinterpret_cast<uint32_t *>(dst);
    for (uint32_t i = threadIdx.x; i < count * words; i += blockDim.x) out[i] = src[i];
}
hipError_t upload_replicas(const Replica *host, uint32_t n, Replica *dev, hipStream_t stream) {
    for (uint32_t i = 0; i < n; i += kUploadPer) {
        ReplicaPack pack;
        uint32_t cnt = n - i < kUploadPer ? n - i : kUploadPer;
        for (uint32_t j = 0; j < cnt; ++j) pack.r[j] = host[i + j];
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, stream, pack, cnt, dev + i);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// The descriptors of spkmc_run_batch_static live in this file-scope device
// array instead of a caller's workspace, so that entry point allocates nothing.
// Each device holds its own copy at its own address, resolved once per device
// (with that device current); host code passes only the resolved address to
// kernels.  Every call on a device shares the array: the descriptors are
// written in full, in stream order, before each launch that reads them.
// ---------------------------------------------------------------------------
constexpr uint32_t kStaticReplicas = 512;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticReplicas * sizeof(Replica)];

uint32_t static_replica_cap() { return kStaticReplicas; }
size_t static_replica_bytes() { return sizeof(scratch); }

hipError_t static_replicas(Replica **out) {
    static std::mutex mu;
    static void *resolved[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!resolved[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        resolved[dev] = ptr;
    }
    *out = reinterpret_cast<Replica *>(resolved[dev]);
    return hipSuccess;
}

// After a captured macro-step: every lattice's next replay starts where this
// one stopped.
__global__ void k_advance_batch(Replica *reps, uint32_t nrep) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrep) reps[i].n0 += reps[i].ncycles;
}

// The descriptors must already be in device memory (dev_reps).
hipError_t launch_batch(const Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, uint32_t lpd,
                        hipStream_t stream) {
    void *kern = select_kernel(h, P, block, true, false, lpd);
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persistent_prep_batch, dim3(n < 256 ? n : 256), dim3(256), 0, stream, dev_reps, n, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const Replica *reps = dev_reps;
    void *args[] = {&reps, &n};
    return hipLaunchCooperativeKernel(kern, dim3(grid), dim3(block), args, 0, stream);
}

// One macro-step as a graph of three kernel nodes: the slot and flag set-up,
// the batch kernel (a cooperative node: every workgroup resident at once, as
// for hipLaunchCooperativeKernel, which stream capture does not take), and the
// descriptor advance.  The descriptors must already be in device memory.
hipError_t capture_batch(Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, uint32_t lpd,
                         hipGraph_t *graph) {
    void *kern = select_kernel(h, P, block, true, false, lpd);
    if (!kern || n == 0) return hipErrorInvalidValue;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    const Replica *creps = dev_reps;
    Replica *mreps = dev_reps;
    uint32_t nn = n;
    int zero = 0;
    void *a_prep[] = {&creps, &nn, &zero};
    void *a_batch[] = {&creps, &nn};
    void *a_adv[] = {&mreps, &nn};
    hipGraphNode_t nprep = nullptr, nbatch = nullptr, nadv = nullptr;
    hipKernelNodeParams kp = {};
    kp.func = reinterpret_cast<void *>(&k_persistent_prep_batch);
    kp.gridDim = dim3(n < 256 ? n : 256);
    kp.blockDim = dim3(256);
    kp.kernelParams = a_prep;
    e = hipGraphAddKernelNode(&nprep, g, nullptr, 0, &kp);
    if (e == hipSuccess) {
        kp.func = kern;
        kp.gridDim = dim3((uint32_t)grid);
        kp.blockDim = dim3((uint32_t)block);
        kp.kernelParams = a_batch;
        e = hipGraphAddKernelNode(&nbatch, g, &nprep, 1, &kp);
    }
    if (e == hipSuccess) {
        hipKernelNodeAttrValue v = {};
        v.cooperative = 1;
        e = hipGraphKernelNodeSetAttribute(nbatch, hipKernelNodeAttributeCooperative, &v);
    }
    if (e == hipSuccess) {
        kp.func = reinterpret_cast<void *>(&k_advance_batch);
        kp.gridDim = dim3((n + 63) / 64);
        kp.blockDim = dim3(64);
        kp.kernelParams = a_adv;
        e = hipGraphAddKernelNode(&nadv, g, &nbatch, 1, &kp);
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    *graph = g;
    return hipSuccess;
}

}  // namespace spkmc
