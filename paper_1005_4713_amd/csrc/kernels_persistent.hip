// kernels_persistent.hip -- the persistent ("PERSISTENT", "INCREMENTAL") engines
// of the gfx950 spkMC library: one cooperative launch runs many cycles (Sec. 3.1
// steps 1-6 with the sublattice steps 4a/4b of Sec. 3.2) over a bit-packed
// lattice; the batch kernel (many lattices in one launch); and the per-cycle
// engine's row kernels (one cycle in two launches, for lattices whose lines do
// not fit the device at once), which share the binning, selection and flip code.
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
#include <string>

#include "spkmc_device.hpp"

namespace spkmc {

namespace {

constexpr int kMaxNbr = 16;                      // neighbour workgroups per direction kept in LDS
constexpr int kMaxGrid = 2048;                   // workgroups of one persistent launch
constexpr int kMaxWgDomains = 256;               // domains of one workgroup
constexpr int kRecBanks = 4;                     // record partial banks
constexpr uint64_t kTimeoutTicks = 200000000ull;  // 2 s of the 100 MHz wall clock
constexpr uint32_t kNoEvent = 0xFFFFFFFFu;

// Device scratch of the persistent engine (its own region of the state).
struct PersistScratch {
    uint64_t *slot;     // 2 x G: R_max of each workgroup, generation bit 63
    uint64_t *flag;     // G: cycles whose flips are complete
    int64_t *recp;      // kRecBanks x G x 3: counter partials (fired, dM, dB) since launch start
    uint64_t *emitted;  // records of this launch appended so far (fixed-bound variant)
};
constexpr uint64_t kScratchWordsPerWg = 2 + 1 + 3 * kRecBanks;

}  // namespace

// One lattice of a persistent launch: its geometry and buffers, its sync
// scratch, the cycles to run, and its range of workgroups in the launch.
struct Replica {
    Geom g;
    PersistScratch xs;
    uint64_t n0, ncycles;
    uint32_t obs_every;
    uint32_t first_wg, G;  // workgroups first_wg .. first_wg + G - 1 run this lattice
    uint32_t pad;
};

namespace {

__device__ __forceinline__ uint32_t ld32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_words2(const uint32_t *p) {  // two consecutive words, 8-byte aligned
    return ld64(reinterpret_cast<const uint64_t *>(p));
}
// Buffer views of the packed spins and of the face copies (byte offsets below
// 2^31 for every size the persistent engine takes), and the cache policy of a
// device-coherent load (sc1).  A load at an offset past the end returns 0: the
// rows of a pass without a line load there, so that every pass issues the same
// loads, unconditionally, and the wait for a pass's words counts only the loads
// issued after them.
constexpr int kCoherent = 16;
struct Views {
    __amdgpu_buffer_rsrc_t A, F;
    int endA, endF;  // sizes in bytes: the offsets that read 0
};
__device__ __forceinline__ Views views_of(const Geom &g) {
    Views v;
    v.endA = (int)(g.N / 8u);
    v.endF = (int)((uint64_t)g.K * 8u * g.fwpo * 4u);
    v.A = __builtin_amdgcn_make_buffer_rsrc((void *)g.A, (short)0, v.endA, 0x00020000);
    v.F = __builtin_amdgcn_make_buffer_rsrc((void *)g.F, (short)0, v.endF, 0x00020000);
    return v;
}
__device__ __forceinline__ uint32_t ld_face(const Views &v, bool valid, uint32_t w) {  // word w of the face copies
    return __builtin_amdgcn_raw_buffer_load_b32(v.F, valid ? (int)(w * 4u) : v.endF, 0, kCoherent);
}
__device__ __forceinline__ void flip_word(uint32_t *p, uint32_t m) {
    (void)__hip_atomic_fetch_xor(p, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// v_bitop3: any boolean function of three words; the immediate is its truth
// table with a = 0xF0, b = 0xCC, c = 0xAA.
constexpr int kXor3 = 0x96, kMaj3 = 0xE8, kAnd3 = 0x80, kSelAC_BnC = 0xE4;  // (a & c) | (b & ~c)
constexpr int kXorOr = 0xBE, kXorNor = 0x41;                                // (a ^ b) | c, ~((a ^ b) | c)
template <int TT>
__device__ __forceinline__ uint32_t bop(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t src) {  // lanes shifted in from outside the row keep old
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint32_t dpp0(uint32_t src) {  // lanes shifted in from outside the row read 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, CTRL, 0xF, 0xF, true);
}
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114,
              kRowShr8 = 0x118, kRowBcast = 0x150;
template <int CTRL>
__device__ __forceinline__ uint32_t bcast(uint32_t v) {  // lane CTRL & 15 of each row to the whole row
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t bcast_lane(uint32_t v, int lane) {  // lane 0..3 of each row (folds when unrolled)
    switch (lane) {
        case 0: return bcast<kRowBcast + 0>(v);
        case 1: return bcast<kRowBcast + 1>(v);
        case 2: return bcast<kRowBcast + 2>(v);
        default: return bcast<kRowBcast + 3>(v);
    }
}

__device__ __forceinline__ uint32_t align_hi(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);  // ({hi, lo} >> s)[31:0]
}

struct DomainCoord {
    int kx, ky, kz;
};
__device__ __forceinline__ DomainCoord dcoord(uint32_t k, int nd) {
    DomainCoord c;
    c.kx = (int)(k % (uint32_t)nd);
    c.ky = (int)((k / (uint32_t)nd) % (uint32_t)nd);
    c.kz = (int)(k / ((uint32_t)nd * (uint32_t)nd));
    return c;
}
__device__ __forceinline__ uint32_t dindex(int kx, int ky, int kz, int nd) {
    return (uint32_t)kx + (uint32_t)nd * ((uint32_t)ky + (uint32_t)nd * (uint32_t)kz);
}
__device__ __forceinline__ int wrapm(int v, int nd) { return v == 0 ? nd - 1 : v - 1; }
__device__ __forceinline__ int wrapp(int v, int nd) { return v + 1 == nd ? 0 : v + 1; }

// The six halo faces of octant (k, s): for each axis the face of the octant of
// colour s ^ (1 << axis) that touches it from below (x1/y1/z1 face) and from
// above (x0/y0/z0 face).  nb holds the six neighbour domains of k
// (-x, +x, -y, +y, -z, +z).
struct HaloFaces {
    uint32_t lo[3];  // word index in F of the face at local coordinate h - 1 of the octant below
    uint32_t hi[3];  // word index in F of the face at local coordinate 0 of the octant above
};
// (32-bit word indices from the uniform base: F holds K * 48 h^2 / 32 words,
// below 2^31 for every supported size)
template <int H>
__device__ __forceinline__ HaloFaces halo_faces(uint32_t k, int s, const uint32_t *nb) {
    HaloFaces hf;
    constexpr uint32_t fw = H * H / 32, fwpo = 6 * fw;  // words per face, per octant
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int bit = (s >> a) & 1;
        const uint32_t c = (uint32_t)(s ^ (1 << a));
        const uint32_t kmi = bit ? k : nb[2 * a], kpi = bit ? nb[2 * a + 1] : k;  // below / above
        // domain indices stay below 2^22 (fewer than 2^34 sites, at least 4096 per
        // domain): a 24-bit multiply
        hf.lo[a] = __umul24(kmi, 8u * fwpo) + c * fwpo + (uint32_t)(2 * a + 1) * fw;
        hf.hi[a] = __umul24(kpi, 8u * fwpo) + c * fwpo + (uint32_t)(2 * a) * fw;
    }
    return hf;
}

// ---------------------------------------------------------------------------
// Per-octant bit planes: spins S and the three bits of n_up for every site.
// ---------------------------------------------------------------------------
template <int H>
struct Planes;
template <>
struct Planes<16> {
    static constexpr int W = 8;  // words per lane
    uint32_t S[W], b0[W], b1[W], b2[W];
};
template <>
struct Planes<8> {
    static constexpr int W = 1;
    uint32_t S[W], b0[W], b1[W], b2[W];
};

// bit-sliced sum of six words: (o2 o1 o0) = number of set inputs at every bit
__device__ __forceinline__ void count6(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f,
                                       uint32_t &o0, uint32_t &o1, uint32_t &o2) {
    uint32_t s1 = bop<kXor3>(a, b, c), c1 = bop<kMaj3>(a, b, c);
    uint32_t s2 = bop<kXor3>(d, e, f), c2 = bop<kMaj3>(d, e, f);
    o0 = s1 ^ s2;
    uint32_t k0 = s1 & s2;
    o1 = bop<kXor3>(c1, c2, k0);
    o2 = bop<kMaj3>(c1, c2, k0);
}

// popcount(x) + acc in one v_bcnt (the compiler otherwise counts into zero and
// sums the counts with extra adds)
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// 13 moments: pop(S), pop(b0), pop(b1), pop(b2), pop(b0b1), pop(b0b2), pop(b1b2)
// and the same six products with S.
__device__ __forceinline__ void moments(uint32_t S, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t (&m)[13]) {
    m[0] = bcnt_acc(S, m[0]);
    m[1] = bcnt_acc(b0, m[1]);
    m[2] = bcnt_acc(b1, m[2]);
    m[3] = bcnt_acc(b2, m[3]);
    m[4] = bcnt_acc(b0 & b1, m[4]);
    m[5] = bcnt_acc(b0 & b2, m[5]);
    m[6] = bcnt_acc(b1 & b2, m[6]);
    m[7] = bcnt_acc(S & b0, m[7]);
    m[8] = bcnt_acc(S & b1, m[8]);
    m[9] = bcnt_acc(S & b2, m[9]);
    m[10] = bcnt_acc(bop<kAnd3>(S, b0, b1), m[10]);
    m[11] = bcnt_acc(bop<kAnd3>(S, b0, b2), m[11]);
    m[12] = bcnt_acc(bop<kAnd3>(S, b1, b2), m[12]);
}

// Histogram (class c = 7 [s = +1] + a) from the moments of an octant of n sites.
// For each spin value the count of sites with exact n_up bit pattern v follows by
// inclusion-exclusion over the products of the bits that are set in v.
__device__ __forceinline__ void hist_from_moments(const uint32_t (&m)[13], uint32_t nsites, uint32_t (&hc)[14]) {
    // up spins: T_U = pop(S & prod U); down spins: total minus up
    int up[7] = {(int)m[0], (int)m[7], (int)m[8], (int)m[9], (int)m[10], (int)m[11], (int)m[12]};
    int all[7] = {(int)nsites, (int)m[1], (int)m[2], (int)m[3], (int)m[4], (int)m[5], (int)m[6]};
    for (int side = 0; side < 2; ++side) {
        int T[7];
        for (int i = 0; i < 7; ++i) T[i] = side == 0 ? up[i] : all[i] - up[i];
        // T[0] = empty product, T[1..3] = b0, b1, b2, T[4] = b0b1, T[5] = b0b2, T[6] = b1b2
        int nv[7];
        nv[0] = T[0] - T[1] - T[2] - T[3] + T[4] + T[5] + T[6];
        nv[1] = T[1] - T[4] - T[5];
        nv[2] = T[2] - T[4] - T[6];
        nv[3] = T[4];
        nv[4] = T[3] - T[5] - T[6];
        nv[5] = T[5];
        nv[6] = T[6];
        for (int v = 0; v < 7; ++v) {
            if (side == 0) hc[7 + v] = (uint32_t)nv[v];  // up spin: aligned = n_up
            else hc[6 - v] = (uint32_t)nv[v];            // down spin: aligned = 6 - n_up
        }
    }
}

// Raw words of one pass, loaded ahead of the pass that uses them.
template <int H>
struct Raw;
template <>
struct Raw<16> {
    uint32_t W[8];            // own plane: word p = rows 2p, 2p + 1
    uint32_t xm, xp, ym, yp;  // words holding this plane's halo rows in the x and y faces
    uint32_t zw;              // lanes 0..7: word l of the face below, lanes 8..15: word l-8 of the face above
};
template <>
struct Raw<8> {
    uint32_t w, xm, xp, yface, zface;
};

// --- h = 16 --------------------------------------------------------------------
// lane l = plane lz; word p holds rows ly = 2p (bits 0..15) and 2p + 1 (bits 16..31).
__device__ __forceinline__ void load16_words(const Geom &g, uint32_t k, int s, bool valid, int l, Raw<16> &r) {
    // the lane's 32 contiguous bytes in two 16-byte device-coherent loads
    const uint32_t a0 = (k * 8u + (uint32_t)s) * 128u + (uint32_t)l * 8u;  // word index, < N / 32
    const Views vw = views_of(g);
#pragma unroll
    for (int p = 0; p < 8; p += 4) {
        const int off = valid ? (int)((a0 + (uint32_t)p) * 4u) : vw.endA;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(vw.A, off, 0, kCoherent);
        r.W[p] = v[0];
        r.W[p + 1] = v[1];
        r.W[p + 2] = v[2];
        r.W[p + 3] = v[3];
    }
}
// the halo words of the axes in the mask `axes` (bit a: axis a)
__device__ __forceinline__ void load16_faces(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                             int axes, Raw<16> &r) {
    const HaloFaces hf = halo_faces<16>(k, s, nb);
    const Views vw = views_of(g);
    // x faces: bit ly + 16 lz -> half-word l; y faces: bit lx + 16 lz -> half-word l
    if (axes & 1) {
        r.xm = ld_face(vw, valid, hf.lo[0] + (l >> 1));
        r.xp = ld_face(vw, valid, hf.hi[0] + (l >> 1));
    }
    if (axes & 2) {
        r.ym = ld_face(vw, valid, hf.lo[1] + (l >> 1));
        r.yp = ld_face(vw, valid, hf.hi[1] + (l >> 1));
    }
    // z faces (bit lx + 16 ly, the layout of a plane), one word per lane
    if (axes & 4) r.zw = ld_face(vw, valid, (l < 8 ? hf.lo[2] : hf.hi[2]) + (l & 7));
}

// zrow: this row's 24 LDS words: face below (8), face above (8), zeros (8).
// MOM: also accumulate the 13 popcount moments of the octant.
template <bool MOM>
__device__ __forceinline__ void compute16(const Raw<16> &r, bool valid, int l, uint32_t *zrow, Planes<16> &P,
                                          uint32_t (&m)[13]) {
    zrow[l] = r.zw;  // the row's own lanes read these back (same wavefront)
    const uint32_t *zlo = zrow + (l == 0 ? 0 : 16), *zhi = zrow + (l == 15 ? 8 : 16);
    const uint32_t sh16 = 16 * (l & 1);
    const uint32_t xm = (r.xm >> sh16) & 0xFFFFu, xp = (r.xp >> sh16) & 0xFFFFu;
    const uint32_t ym = (r.ym >> sh16) & 0xFFFFu, yp = (r.yp >> sh16) & 0xFFFFu;
    // x halo bits: word p needs xm bits 2p, 2p+1 at bits 0, 16 and xp bits 2p, 2p+1 at 15, 31
    const uint32_t Tm = xm | (xm << 15), Tp = xp | (xp << 15);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const uint32_t w = r.W[p];
        uint32_t nxm = bop<kSelAC_BnC>(w << 1, Tm >> (2 * p), 0xFFFEFFFEu);
        uint32_t nxp = bop<kSelAC_BnC>(w >> 1, Tp << (15 - 2 * p), 0x7FFF7FFFu);
        uint32_t nym = p == 0 ? ((w << 16) | ym) : align_hi(w, r.W[p - 1], 16);
        uint32_t nyp = p == 7 ? align_hi(yp, w, 16) : align_hi(r.W[p + 1], w, 16);
        // plane lz -+ 1; the first and last lane take the face word instead
        uint32_t nzm = dpp0<kRowShr1>(w) | zlo[p];
        uint32_t nzp = dpp0<kRowShl1>(w) | zhi[p];
        uint32_t o0, o1, o2;
        count6(nxm, nxp, nym, nyp, nzm, nzp, o0, o1, o2);
        P.S[p] = w;
        P.b0[p] = o0;
        P.b1[p] = o1;
        P.b2[p] = o2;
        if (MOM) moments(w, o0, o1, o2, m);  // invalid rows hold zeros
    }
}

// --- h = 8 ---------------------------------------------------------------------
// lane l = 2 lz + p holds word l: rows ly = 4p .. 4p + 3 of plane lz, 8 bits each.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) {  // bits 0..3 -> bits 0, 8, 16, 24
    return (nib * 0x00204081u) & 0x01010101u;
}
__device__ __forceinline__ void load8_words(const Geom &g, uint32_t k, int s, bool valid, int l, Raw<8> &r) {
    const Views vw = views_of(g);
    const int off = valid ? (int)(((k * 8u + (uint32_t)s) * 16u + (uint32_t)l) * 4u) : vw.endA;
    r.w = __builtin_amdgcn_raw_buffer_load_b32(vw.A, off, 0, kCoherent);
}
__device__ __forceinline__ void load8_faces(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                            int axes, Raw<8> &r) {
    const int lz = l >> 1, p = l & 1;
    const HaloFaces hf = halo_faces<8>(k, s, nb);
    const Views vw = views_of(g);
    // x faces: bit ly + 8 lz; rows 4p..4p+3 of plane lz = bits 4l .. 4l + 3
    if (axes & 1) {
        r.xm = ld_face(vw, valid, hf.lo[0] + (l >> 3));
        r.xp = ld_face(vw, valid, hf.hi[0] + (l >> 3));
    }
    // y faces: bit lx + 8 lz = byte lz; the lowest row of p = 0 needs the face below,
    // the highest row of p = 1 the face above
    if (axes & 2) r.yface = ld_face(vw, valid, (p == 0 ? hf.lo[1] : hf.hi[1]) + (lz >> 2));
    // z faces: bit lx + 8 ly, word p covers rows 4p .. 4p + 3; the inner planes read 0
    if (axes & 4) r.zface = ld_face(vw, valid && (lz == 0 || lz == 7), (lz == 0 ? hf.lo[2] : hf.hi[2]) + p);
}

template <bool MOM>
__device__ __forceinline__ void compute8(const Raw<8> &r, bool valid, int l, uint32_t *, Planes<8> &P,
                                         uint32_t (&m)[13]) {
    int lz = l >> 1, p = l & 1;
    const uint32_t w = r.w;
    const uint32_t xm = (r.xm >> (4 * (l & 7))) & 0xFu, xp = (r.xp >> (4 * (l & 7))) & 0xFu;
    const uint32_t yface = (r.yface >> (8 * (lz & 3))) & 0xFFu;
    uint32_t nxm = bop<kSelAC_BnC>(w << 1, spread4(xm), 0xFEFEFEFEu);
    uint32_t nxp = bop<kSelAC_BnC>(w >> 1, spread4(xp) << 7, 0x7F7F7F7Fu);
    uint32_t below = dpp0<kRowShr1>(w);  // word l - 1 (row 4p - 1 when p = 1)
    uint32_t above = dpp0<kRowShl1>(w);  // word l + 1 (row 4p + 4 when p = 0)
    uint32_t nym = p ? align_hi(w, below, 24) : ((w << 8) | yface);
    uint32_t nyp = p ? ((yface << 24) | (w >> 8)) : align_hi(above, w, 8);
    uint32_t nzm = dpp<kRowShr2>(r.zface, w);  // plane lz - 1 (lanes 0, 1 keep the face below)
    uint32_t nzp = dpp<kRowShl2>(r.zface, w);  // plane lz + 1 (lanes 14, 15 keep the face above)
    uint32_t o0, o1, o2;
    count6(nxm, nxp, nym, nyp, nzm, nzp, o0, o1, o2);
    P.S[0] = w;
    P.b0[0] = o0;
    P.b1[0] = o1;
    P.b2[0] = o2;
    if (MOM) moments(w, o0, o1, o2, m);  // invalid rows hold zeros
}

template <int H>
__device__ __forceinline__ void load_words(const Geom &g, uint32_t k, int s, bool valid, int l, Raw<H> &r) {
    if constexpr (H == 16) load16_words(g, k, s, valid, l, r);
    else load8_words(g, k, s, valid, l, r);
}
template <int H>
__device__ __forceinline__ void load_faces(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                           int axes, Raw<H> &r) {
    if constexpr (H == 16) load16_faces(g, k, s, valid, l, nb, axes, r);
    else load8_faces(g, k, s, valid, l, nb, axes, r);
}
template <int H>
__device__ __forceinline__ void load_octant(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                            Raw<H> &r) {
    load_words<H>(g, k, s, valid, l, r);
    load_faces<H>(g, k, s, valid, l, nb, 7, r);
}
template <int H, bool MOM>
__device__ __forceinline__ void compute_octant(const Raw<H> &r, bool valid, int l, uint32_t *zrow, Planes<H> &P,
                                               uint32_t (&m)[13]) {
    if constexpr (H == 16) compute16<MOM>(r, valid, l, zrow, P, m);
    else compute8<MOM>(r, valid, l, zrow, P, m);
}

// ---------------------------------------------------------------------------
// Incremental class histograms (the class changes a flip causes, step 6)
// ---------------------------------------------------------------------------
// Class of a site from its spin (1 = up) and its number of up neighbours: an up
// spin is aligned with its up neighbours, a down spin with the others.
__device__ __forceinline__ int site_class(uint32_t up, int nup) { return up ? 7 + nup : 6 - nup; }

// Packed counts: class c in the 16-bit half (c & 1) of word c >> 1 (h^3 <= 4096).
__device__ __forceinline__ uint32_t hcount(const uint32_t *hp, int c) {
    return (hp[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
}
__device__ __forceinline__ void hadd(uint32_t *hp, int c, int v) {  // a count never drops below 0
    atomicAdd(&hp[c >> 1], (uint32_t)v << (16 * (c & 1)));
}
// A site leaves class c_old for c_new.
__device__ __forceinline__ void hmove(uint32_t *hp, int c_old, int c_new) {
    hadd(hp, c_old, -1);
    hadd(hp, c_new, 1);
}

// Where site (x, y, z) of an octant sits in the class planes of a row: lane,
// word and bit (h = 16: lane z, word y / 2; h = 8: lane 2 z + y / 4, one word).
template <int H>
__device__ __forceinline__ void plane_loc(int x, int y, int z, int &lane, int &word, int &bit) {
    if constexpr (H == 16) {
        lane = z;
        word = y >> 1;
        bit = x + 16 * (y & 1);
    } else {
        lane = 2 * z + (y >> 2);
        word = 0;
        bit = x + 8 * (y & 3);
    }
}

// Spin (1 = up) of the site at domain-local coordinates T (each in [-2h, 4h))
// of the domain at c; coordinates outside [0, 2h) belong to the periodic
// neighbour domain.  Sets the domain and octant of the site.
template <int H>
__device__ __forceinline__ uint32_t spin_at(const Geom &g, DomainCoord c, const int (&T)[3], uint32_t &k, int &o) {
    int kc[3] = {c.kx, c.ky, c.kz}, X[3];
    o = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        X[a] = T[a];
        if (X[a] < 0) {
            X[a] += 2 * H;
            kc[a] = wrapm(kc[a], g.nd);
        } else if (X[a] >= 2 * H) {
            X[a] -= 2 * H;
            kc[a] = wrapp(kc[a], g.nd);
        }
        o |= (X[a] >= H) << a;
    }
    k = dindex(kc[0], kc[1], kc[2], g.nd);
    const uint32_t q = (uint32_t)((X[0] & (H - 1)) + H * ((X[1] & (H - 1)) + H * (X[2] & (H - 1))));
    const uint32_t word = (k * 8u + (uint32_t)o) * (uint32_t)(H * H * H / 32) + (q >> 5);  // < N / 32 < 2^31
    return (ld32(&g.A[word]) >> (q & 31)) & 1u;
}

// Class changes pushed to a domain of another workgroup: per (domain, octant,
// spin) one 64-bit word holding 7 signed base-512 digits, digit a = the net
// change of the class with aligned count a.  Pushes are atomic adds; the owner
// takes the word with an exchange and recovers the digits (each stays within
// +-255: at most one push reaches an octant per cycle, and every octant is
// folded at least once per kFoldAll cycles).
constexpr uint64_t kFoldAll = 64;
__device__ __forceinline__ uint64_t digit_move(int a_old, int a_new) {
    return (1ull << (9 * a_new)) - (1ull << (9 * a_old));
}
// Fold a taken word into the packed counts of spin half `up`; false if the
// word was not a sum of in-range digits.
__device__ __forceinline__ bool fold_word(uint64_t v, int up, uint32_t *hp) {
    int64_t V = (int64_t)v;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int64_t dig = ((V & 511) ^ 256) - 256;
        V = (V - dig) >> 9;
        if (dig) hadd(hp, 7 * up + i, (int)dig);
    }
    return V == 0;
}

// Inclusive prefix sum over the 16 lanes of a DPP row (lane 15 ends with the
// row total): four shifted adds, lanes shifted in from outside the row add 0.
__device__ __forceinline__ uint32_t row_scan(uint32_t v) {
    v += dpp0<kRowShr1>(v);
    v += dpp0<kRowShr2>(v);
    v += dpp0<kRowShr4>(v);
    v += dpp0<kRowShr8>(v);
    return v;
}

// position of the r-th (0-based) set bit of m (r < popcount(m)), by halving
__device__ __forceinline__ int nth_set_bit(uint32_t m, uint32_t r) {
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        uint32_t c = __builtin_popcount(m & ((1u << w) - 1u));
        if (r >= c) {
            r -= c;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// Maximum of a non-negative double over the wavefront, returned in lane 63:
// DPP shifts within each row (lanes from outside read 0), then the last lane of
// each row carried into the rows above.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
__device__ __forceinline__ double wave_max_nonneg(double v) {
    v = fmax(v, dpp_f64<kRowShr1, 0xF>(v));
    v = fmax(v, dpp_f64<kRowShr2, 0xF>(v));
    v = fmax(v, dpp_f64<kRowShr4, 0xF>(v));
    v = fmax(v, dpp_f64<kRowShr8, 0xF>(v));
    v = fmax(v, dpp_f64<kRowBcast15, 0xA>(v));
    v = fmax(v, dpp_f64<kRowBcast31, 0xC>(v));
    return v;
}

// --- pieces of a cycle shared by the persistent kernels and the two-launch
// (per-cycle) row kernels

// One row's class for a target: lane c of the row tests class c against the
// line's running sums acc (-1: the null event).
__device__ __forceinline__ int row_class(const double *acc, bool valid, double target, int l, int row) {
    const bool hit = valid && l < 14 && target < acc[l < 14 ? l : 13];
    const uint64_t bal = __ballot(hit);
    const uint32_t rowbits = (uint32_t)(bal >> (16 * (row & 3))) & 0xFFFFu;
    return rowbits ? __builtin_ctz(rowbits) : -1;
}

// The event of a row for class cs with ncs sites: the j-th site of the class in
// canonical order (j from the uniform uz), written into the row's selection slot
// as (cs << 12) | q, or kNoEvent.  Every lane of the row takes part.
template <int H>
__device__ __forceinline__ void select_site(const Planes<H> &pl, int cs, uint32_t ncs, uint32_t uz, int l,
                                            uint32_t *slot, DevState *st) {
    constexpr int WPL = Planes<H>::W;
    if (l == 0) *slot = kNoEvent;
    const uint32_t j = cs >= 0 ? mul_index(uz, ncs) : 0u;
    // class cs as (spin, n_up pattern): up spin (cs >= 7): n_up = cs - 7; down
    // spin: n_up = 6 - cs.  A row without an event never uses its masks.
    const int up = cs >= 7, v = up ? cs - 7 : 6 - cs;
    const uint32_t ps = up ? 0xFFFFFFFFu : 0u;  // the pattern each plane must equal
    const uint32_t p0 = (v & 1) ? 0xFFFFFFFFu : 0u, p1 = (v & 2) ? 0xFFFFFFFFu : 0u;
    const uint32_t p2 = (v & 4) ? 0xFFFFFFFFu : 0u;
    uint32_t mk[WPL], cum[WPL];
    uint32_t cnt = 0;
#pragma unroll
    for (int p = 0; p < WPL; ++p) {
        // sites of class cs: no plane differs from its pattern; (a ^ b) | c per step
        uint32_t d = pl.S[p] ^ ps;
        d = bop<kXorOr>(pl.b0[p], p0, d);
        d = bop<kXorOr>(pl.b1[p], p1, d);
        mk[p] = bop<kXorNor>(pl.b2[p], p2, d);
        cnt = bcnt_acc(mk[p], cnt);
        cum[p] = cnt;  // running count over the lane's words
    }
    // inclusive prefix over the 16 lanes of the row (canonical order = lane order)
    const uint32_t incl = row_scan(cnt);
    const uint32_t excl = incl - cnt;
    if (cs >= 0 && l == 15 && j >= incl) atomicOr(&st->error, kErrSelect);  // counts disagree with masks
    if (cs >= 0 && j >= excl && j < incl) {
        // the word holding the target: as many words as have running counts not
        // above its rank; then its rank inside that word
        const uint32_t r0 = j - excl;
        uint32_t wsel = 0;
#pragma unroll
        for (int p = 0; p + 1 < WPL; ++p) wsel += cum[p] <= r0 ? 1u : 0u;
        uint32_t before = 0, msk = mk[0];
#pragma unroll
        for (int p = 1; p < WPL; ++p)
            if (wsel == (uint32_t)p) {
                before = cum[p - 1];
                msk = mk[p];
            }
        const uint32_t q = (uint32_t)(l * WPL) * 32 + wsel * 32 + (uint32_t)nth_set_bit(msk, r0 - before);
        *slot = ((uint32_t)cs << 12) | q;  // after lane 0's store, same wavefront
    }
}

// Flip site q of octant (k, so): its spin word and the face copies it appears in.
template <int H>
__device__ __forceinline__ void flip_site(const Geom &g, uint32_t k, int so, uint32_t q) {
    constexpr uint32_t wpo = H * H * H / 32, fwpo = 6 * H * H / 32;
    flip_word(g.A + ((uint64_t)k * 8 + (uint32_t)so) * wpo + (q >> 5), 1u << (q & 31));
    const uint32_t lx = q % H, ly = (q / H) % H, lz = q / (H * H);
    uint32_t *F = g.F + ((uint64_t)k * 8 + (uint32_t)so) * fwpo;
    constexpr uint32_t e = H - 1, h2 = H * H;
    if (lx == 0) { uint32_t b = ly + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
    if (lx == e) { uint32_t b = h2 + ly + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
    if (ly == 0) { uint32_t b = 2 * h2 + lx + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
    if (ly == e) { uint32_t b = 3 * h2 + lx + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
    if (lz == 0) { uint32_t b = 4 * h2 + lx + H * ly; flip_word(F + (b >> 5), 1u << (b & 31)); }
    if (lz == e) { uint32_t b = 5 * h2 + lx + H * ly; flip_word(F + (b >> 5), 1u << (b & 31)); }
}

// wall clock (100 MHz) for bounded waits
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

}  // namespace

// Workgroup-shared state of the persistent kernel.
struct PersistShared {
    double r[14];                      // rate table
    uint32_t mom[kMaxWgDomains][13];   // per domain: the 13 popcount moments of its active octant
    uint32_t hist[kMaxWgDomains][14];  // per domain: class histogram (re-binning engine)
    uint32_t histp[kMaxWgDomains][8][7];  // per domain and octant: packed class counts (incremental engine)
    double acc[kMaxWgDomains][14];     // per domain: running FP64 sums of the frequency line
    double rk[kMaxWgDomains];
    uint32_t zbuf[64][24];             // per row: z face words below (8), above (8), zeros (8)
    uint32_t nbdom[kMaxWgDomains][6];  // per domain: the neighbour domains -x, +x, -y, +y, -z, +z
    uint32_t selq[kMaxWgDomains];      // per row: (class << 12) | site q of its event, or kNoEvent
    double rpred[8];                   // per colour: the last R_max seen (the prediction)
    double rmax;
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

// Sum the partials of the oldest pending record over all workgroups (one
// wavefront) and append the record.  The caller guarantees every workgroup has
// stored them.
template <class SH>
__device__ __forceinline__ void emit_record(const Geom &g, const PersistScratch &xs, SH &sh, uint32_t G,
                                            int lane, uint64_t n0, uint64_t fired0, uint64_t nulls0, int64_t M0,
                                            int64_t B0) {
    const uint32_t slot = sh.pend_head % kRecBanks;
    const int64_t *rp = xs.recp + (uint64_t)sh.pend_bank[slot] * G * 3;
    long long F = 0, dM = 0, dB = 0;
    for (uint32_t w = (uint32_t)lane; w < G; w += 64) {
        F += (long long)ld64((const uint64_t *)&rp[3 * w]);
        dM += (long long)ld64((const uint64_t *)&rp[3 * w + 1]);
        dB += (long long)ld64((const uint64_t *)&rp[3 * w + 2]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        F += __shfl_xor(F, o);
        dM += __shfl_xor(dM, o);
        dB += __shfl_xor(dB, o);
    }
    if (lane == 0) {
        const uint64_t cyc = sh.pend_cycle[slot];
        spkmc_record r;
        r.cycle = cyc;
        r.fired = fired0 + (uint64_t)F;
        r.nulls = nulls0 + (uint64_t)g.K * g.lpd * (cyc - n0) - (uint64_t)F;
        r.t = sh.pend_t[slot];
        r.M = M0 + dM;
        r.B = B0 + dB;
        DevState *st = g.st;
        g.rec[st->rec_count % g.rec_cap] = r;
        st->rec_count += 1;
        sh.pend_head += 1;
    }
}

// Wait until the neighbour workgroups in direction dir (all six directions for
// dir < 0) have completed `upto` cycles; false on a timeout (error set).
template <int BLOCK, class SH>
__device__ __forceinline__ bool wait_neighbours(const PersistScratch &xs, DevState *st, SH &sh, uint32_t G,
                                                int dir, uint64_t upto) {
    const int tid = threadIdx.x;
    for (int d = dir < 0 ? 0 : dir; d < (dir < 0 ? 6 : dir + 1); ++d) {
        const bool all = sh.nbr_cnt[d] > kMaxNbr;
        const uint32_t cnt = all ? G : sh.nbr_cnt[d];
        for (uint32_t i = tid; i < cnt; i += BLOCK) {
            const uint32_t w = all ? i : sh.nbr[d][i];
            const uint64_t start = now_ticks();
            while (ld64(&xs.flag[w]) < upto) {
                __builtin_amdgcn_s_sleep(1);
                if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                    atomicOr(&st->error, kErrFlagTimeout);
                    sh.abort = 1;
                    break;
                }
            }
        }
    }
    __syncthreads();
    return !sh.abort;
}

// Bin octant o of every domain of the workgroup (the 13 moments of each row, then
// its histogram) into the packed counts of that octant.
template <int H, int P, int BLOCK>
__device__ __forceinline__ void bin_all(const Geom &g, uint32_t kbase, uint32_t nvalid, int o, PersistShared &sh) {
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
template <int H, int P, int BLOCK, bool INC, int LPD>
__device__ __forceinline__ void persistent_body(const Replica &R, const uint32_t gid, PersistShared &sh) {
    const Geom &g = R.g;
    const PersistScratch &xs = R.xs;
    const uint64_t n0 = R.n0, ncycles = R.ncycles;
    const uint32_t obs_every = R.obs_every;
    constexpr int nthr = BLOCK;
    constexpr int rows = BLOCK / 16;        // domains per pass
    const int tid = threadIdx.x;
    const int row = tid >> 4, l = tid & 15;  // DPP row and lane inside it
    const uint32_t G = R.G;
    const uint32_t D = (uint32_t)(rows * P);
    // rows run frequency lines: one per domain, or (two colours) the four active
    // octants of each domain, lines 4k .. 4k + 3 of domain k
    const uint32_t lpd = LPD ? (uint32_t)LPD : g.lpd, NL = g.K * lpd;  // LPD = 0: read at run time
    const uint32_t kbase = gid * D;  // first line of the workgroup
    const uint32_t nvalid = kbase >= NL ? 0u : (NL - kbase < D ? NL - kbase : D);
    auto line_dom = [lpd](uint32_t line) { return lpd == 1 ? line : line >> 2; };
    auto line_oct = [lpd](uint32_t line, int colour) {
        return lpd == 1 ? colour : two_colour_octant(colour, line & 3u);
    };
    const bool recorder = gid == 0;
    const uint64_t n_end = n0 + ncycles;

    // neighbour workgroups per direction (0: -x, 1: +x, 2: -y, 3: +y, 4: -z, 5: +z)
    for (uint32_t i = tid; i < 6 * (kMaxGrid / 32); i += nthr) (&sh.nbr_bits[0][0])[i] = 0;
    if (tid == 0) {
        sh.abort = 0;
        sh.pend_head = sh.pend_tail = 0;
    }
    if (tid < 8) sh.rpred[tid] = 0.0;  // no prediction yet
    if (tid < 14) sh.r[tid] = g.r[tid];
    if (l < 8) sh.zbuf[row][16 + l] = 0;
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
    if (tid < 6) {
        uint32_t cnt = 0;
        for (uint32_t w = 0; w < G; ++w)
            if ((sh.nbr_bits[tid][w >> 5] >> (w & 31)) & 1u) {
                if (cnt < kMaxNbr) sh.nbr[tid][cnt] = w;
                ++cnt;
            }
        sh.nbr_cnt[tid] = cnt;
    }
    __syncthreads();

    // INC: the histograms of all eight octants, from the spins at launch start
    // (no workgroup flips before every workgroup has published its first R_max)
    if constexpr (INC) {
#pragma unroll 1
        for (int o = 0; o < 8; ++o) bin_all<H, P, BLOCK>(g, kbase, nvalid, o, sh);
    }

    DevState *st = g.st;
    // launch-start totals (read before any workgroup can publish its first slot,
    // hence before any workgroup can fold its own totals in at the end)
    const uint64_t fired0 = st->fired, nulls0 = st->nulls;
    const int64_t M0 = st->M, B0 = st->B;
    double t = st->t;  // every workgroup advances the same clock
    long long myF = 0, mydM = 0, mydB = 0;  // this thread's share since launch start
    uint32_t rec_index = 0;                  // records produced in this launch
    int prev_colour = -1;
    const bool bound = (g.variant & SPKMC_VARIANT_RMAX_BOUND) != 0;   // re-binning engine only
    const bool rmax_all = INC && (g.variant & SPKMC_VARIANT_RMAX_ALL);  // incremental engine only
    // -ln u of the coming cycle's clock step
    double lnu = -log(cycle_draw(g.seed, n0, lpd == 4).ut);
    // the cycle after which the next observation record falls due
    uint64_t next_rec = obs_every ? (n0 / obs_every + 1) * obs_every : ~0ull;

    for (uint64_t n = n0; n < n_end; ++n) {
        CycleDraw cd = cycle_draw(g.seed, n, lpd == 4);
        const int s = cd.colour;  // the octant (eight colours) or the parity (two)

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
                // row totals (at most h^3 <= 4096 each), two to a word for the scan
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
            __syncthreads();
            // step 1: histogram and frequency line of every domain of the workgroup,
            // running sums kept for the selection (the same sums in the same order)
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
        // lane pp of each row draws for the row's line of pass pp
        U4 dw;
        {
            const uint32_t kd = kbase + (uint32_t)((l < P ? l : 0) * rows + row);
            dw = philox10((uint32_t)n, (uint32_t)(n >> 32), line_dom(kd), (uint32_t)line_oct(kd, s), g.seed);
        }
        // sites of class c on line ld
        auto line_count = [&](uint32_t ld, int c) -> uint32_t {
            return INC ? hcount(sh.histp[ld][s], c) : sh.hist[ld][c];
        };
        uint32_t cpred = 0;  // per pass: predicted class + 1, five bits each
        {
            const double Rspec = bound ? g.rbound : sh.rpred[s];
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
                const int cs = row_class(sh.acc[ld], ld < nvalid, unit53(ux, uy) * Rspec, l, row);
                cpred |= (uint32_t)(cs + 1) << (5 * pp);
                select_site<H>(pl[pp], cs, cs >= 0 ? line_count(ld, cs) : 0u, uz, l, &sh.selq[ld], st);
            }
        }

        if (tid < 64 && !bound) {
            // workgroup 0 sums a record stored two or more cycles ago while it waits
            if (recorder && sh.pend_head != sh.pend_tail && sh.pend_cycle[sh.pend_head % kRecBanks] + 2 <= n + 1)
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
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
        const double Rmax = bound ? g.rbound : sh.rmax;

        if (!bound) {
            // the true R_max: rows whose class differs select again
            if (tid == 0) sh.rpred[s] = Rmax;
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t ld = (uint32_t)(pp * rows + row);
                const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
                const int cs = row_class(sh.acc[ld], ld < nvalid, unit53(ux, uy) * Rmax, l, row);
                if ((uint32_t)(cs + 1) != ((cpred >> (5 * pp)) & 31u))
                    select_site<H>(pl[pp], cs, cs >= 0 ? line_count(ld, cs) : 0u, uz, l, &sh.selq[ld], st);
            }
        }
        __syncthreads();
        // --- the flips of this cycle
        // one thread per row with an event; incremental engine: three threads per
        // such row, one per axis, each moving the
        // classes of the flipped site's two neighbours along its axis; the first
        // also flips the site (spin word and face copies) and moves its class
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
            flip_site<H>(g, k, so, q);
            myF += 1;
            mydM += cs >= 7 ? -2 : 2;              // the class carries the old spin
            mydB += 12 - 4 * (long long)(cs % 7);  // and its aligned count
        }

        // this thread's flips complete (its only memory operations in flight)
        __builtin_amdgcn_s_waitcnt(0);

        // --- step 5: the clock, identical in every workgroup
        {
            double dt = lnu / ((lpd == 4 ? 2.0 : 8.0) * Rmax);
            t = t + dt;
        }
        lnu = -log(cycle_draw(g.seed, n + 1, lpd == 4).ut);
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
                    // end of the launch: fold this workgroup's share into the totals
                    atomicAdd((unsigned long long *)&st->fired, (unsigned long long)F);
                    atomicAdd((unsigned long long *)&st->nulls,
                              (unsigned long long)((long long)nvalid * (long long)ncycles - F));
                    atomicAdd((unsigned long long *)&st->M, (unsigned long long)dM);
                    atomicAdd((unsigned long long *)&st->B, (unsigned long long)dB);
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
            if (record || last) __builtin_amdgcn_s_waitcnt(0);
            st64(&xs.flag[gid], n + 1);
        }
        if (bound && record && !last) {  // uniform over the workgroup
            if (recorder && tid < 64) {
                // fixed bound: workgroup 0 appends the record as soon as every
                // workgroup has completed the cycle (its own flag is already out)
                const uint64_t start = now_ticks();
                bool ok = true;
                for (uint32_t w = tid; w < G && ok; w += 64)
                    while (ld64(&xs.flag[w]) < n + 1) {
                        __builtin_amdgcn_s_sleep(1);
                        if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                            atomicOr(&st->error, kErrFlagTimeout);
                            sh.abort = 1;
                            ok = false;
                            break;
                        }
                    }
                if (__all(ok)) {
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
        if (tid < 64 && !sh.abort) {
            uint64_t start = now_ticks();
            for (uint32_t w = tid; w < G; w += 64)
                while (ld64(&xs.flag[w]) < n_end) {
                    __builtin_amdgcn_s_sleep(1);
                    if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                        atomicOr(&st->error, kErrFlagTimeout);
                        sh.abort = 1;
                        break;
                    }
                }
        }
        __syncthreads();
        if (tid < 64 && !sh.abort) {
            while (sh.pend_head != sh.pend_tail) {
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
                __builtin_amdgcn_wave_barrier();
            }
            if (tid == 0) {
                st->t = t;
                st->cycle = n_end;
                if (obs_every && (n_end % obs_every) == 0 && g.rec_cap) {
                    spkmc_record r;
                    r.cycle = n_end;
                    r.fired = ld64(&st->fired);
                    r.nulls = ld64(&st->nulls);
                    r.t = t;
                    r.M = (int64_t)ld64((const uint64_t *)&st->M);
                    r.B = (int64_t)ld64((const uint64_t *)&st->B);
                    g.rec[st->rec_count % g.rec_cap] = r;
                    st->rec_count += 1;
                }
            }
        }
    }
}

// One lattice: the descriptor by value; LPD, the frequency lines per domain (1
// or 4), fixed at compile time so that every line of a pass shares its octant.
template <int H, int P, int BLOCK, bool INC, int LPD>
__global__ void __launch_bounds__(BLOCK) k_persistent(Replica R) {
    __shared__ PersistShared sh;
    persistent_body<H, P, BLOCK, INC, LPD>(R, blockIdx.x, sh);
}

// ---------------------------------------------------------------------------
// The per-cycle engine's row kernels (PACKED, octant edge 8 or 16): one cycle in
// two launches, for lattices of any size.  k_rows_bin bins every line with the
// persistent kernel's rows and passes (step 1) and takes the maximum (step 2)
// into st->rmax[0]; k_rows_select derives the class planes again, draws,
// selects and flips (steps 3, 4, 4b; step 6 is the launch boundary); the
// per-cycle k_finalize keeps the clock, the counters and the records (step 5).
constexpr int kRowsPasses = 4;  // passes of the row kernels (128 or 256 lines per workgroup)

struct RowsShared {
    uint32_t zbuf[64][24];             // per row: z face words below (8), above (8), zeros (8)
    uint32_t nbdom[kMaxWgDomains][6];  // per line: its domain's six neighbour domains
    double acc[kMaxWgDomains][14];     // per line: running FP64 sums of the frequency line
    uint32_t hist[kMaxWgDomains][14];  // per line: class counts
    uint32_t selq[kMaxWgDomains];      // per line: (class << 12) | site q, or kNoEvent
    unsigned long long wmax;           // the workgroup's largest line (FP64 bits)
    long long red[3][16];
};

template <int H, int BLOCK, int LPD, int PASSES>
struct RowsGeometry {
    static constexpr int rows = BLOCK / 16, P = PASSES;
    static constexpr uint32_t D = rows * P;  // lines of one workgroup
    const Geom &g;
    uint32_t lpd, kbase, nvalid;
    __device__ RowsGeometry(const Geom &g_) : g(g_) {
        lpd = LPD ? (uint32_t)LPD : g.lpd;
        const uint32_t NL = g.K * lpd;
        kbase = blockIdx.x * D;
        nvalid = kbase >= NL ? 0u : (NL - kbase < D ? NL - kbase : D);
    }
    __device__ uint32_t dom(uint32_t line) const { return lpd == 1 ? line : line >> 2; }
    __device__ int oct(uint32_t line, int colour) const {
        return lpd == 1 ? colour : two_colour_octant(colour, line & 3u);
    }
    // the neighbour domains of every line of the workgroup, into LDS
    __device__ void neighbours(uint32_t (*nbdom)[6]) const {
        for (uint32_t i = threadIdx.x; i < nvalid * 6; i += BLOCK) {
            const uint32_t ldm = i / 6;
            const int dir = (int)(i % 6), a = dir >> 1;
            const DomainCoord c = dcoord(dom(kbase + ldm), g.nd);
            int kc[3] = {c.kx, c.ky, c.kz};
            kc[a] = (dir & 1) ? wrapp(kc[a], g.nd) : wrapm(kc[a], g.nd);
            nbdom[ldm][dir] = dindex(kc[0], kc[1], kc[2], g.nd);
        }
    }
};

template <int H, int BLOCK, int LPD, int PASSES>
__global__ void __launch_bounds__(BLOCK) k_rows_bin(Geom g, uint64_t n) {
    __shared__ RowsShared sh;
    using RG = RowsGeometry<H, BLOCK, LPD, PASSES>;
    constexpr int rows = RG::rows, P = RG::P;
    const RG rg(g);
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
    const int s = cycle_draw(g.seed, n, rg.lpd == 4).colour;
    rg.neighbours(sh.nbdom);
    if (tid == 0) sh.wmax = 0;
    if (l < 8) sh.zbuf[row][16 + l] = 0;
    __syncthreads();
    Raw<H> raw[P];
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < rg.nvalid;
        load_octant<H>(g, rg.dom(rg.kbase + ld), rg.oct(rg.kbase + ld, s), valid, l, sh.nbdom[valid ? ld : 0],
                       raw[pp]);
    }
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < rg.nvalid;
        Planes<H> pl;
        uint32_t m[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) m[i] = 0;
        compute_octant<H, true>(raw[pp], valid, l, sh.zbuf[row], pl, m);
        uint32_t mp[7];  // row totals, two to a word
#pragma unroll
        for (int i = 0; i < 6; ++i) mp[i] = row_scan(m[2 * i] | (m[2 * i + 1] << 16));
        mp[6] = row_scan(m[12]);
        if (l == 15 && valid) {
            uint32_t mm[13], hc[14];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                mm[2 * i] = mp[i] & 0xFFFFu;
                mm[2 * i + 1] = mp[i] >> 16;
            }
            mm[12] = mp[6];
            hist_from_moments(mm, (uint32_t)(H * H * H), hc);
            const uint64_t f = rg.kbase + ld;
            for (int c = 0; c < 16; ++c) g.hist[f * 16 + c] = c < 14 ? hc[c] : 0u;
            const double Rk = line_total(hc, g.r);
            g.Rk[f] = Rk;
            atomicMax(&sh.wmax, (unsigned long long)double_to_bits(Rk));
        }
    }
    __syncthreads();
    if (tid == 0 && rg.nvalid && !(g.variant & SPKMC_VARIANT_RMAX_BOUND))
        atomicMax((unsigned long long *)&g.st->rmax[0], sh.wmax);
}

template <int H, int BLOCK, int LPD, int PASSES>
__global__ void __launch_bounds__(BLOCK) k_rows_select(Geom g, uint64_t n) {
    __shared__ RowsShared sh;
    using RG = RowsGeometry<H, BLOCK, LPD, PASSES>;
    constexpr int rows = RG::rows, P = RG::P;
    constexpr uint32_t D = RG::D;
    const RG rg(g);
    const int tid = threadIdx.x, row = tid >> 4, l = tid & 15;
    const int s = cycle_draw(g.seed, n, rg.lpd == 4).colour;
    const double Rmax = (g.variant & SPKMC_VARIANT_RMAX_BOUND) ? g.rbound : bits_to_double(g.st->rmax[0]);
    rg.neighbours(sh.nbdom);
    if (l < 8) sh.zbuf[row][16 + l] = 0;
    // the counts of every line and their running sums, in the order of step 1
    for (uint32_t i = tid; i < D; i += BLOCK) {
        double a = 0.0;
        for (int c = 0; c < 14; ++c) {
            const uint32_t cnt = i < rg.nvalid ? g.hist[(uint64_t)(rg.kbase + i) * 16 + c] : 0u;
            sh.hist[i][c] = cnt;
            double term = (double)cnt * g.r[c];
            a = a + term;
            sh.acc[i][c] = a;
        }
    }
    __syncthreads();
    Raw<H> raw[P];
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < rg.nvalid;
        load_octant<H>(g, rg.dom(rg.kbase + ld), rg.oct(rg.kbase + ld, s), valid, l, sh.nbdom[valid ? ld : 0],
                       raw[pp]);
    }
    // lane pp of each row draws for the row's line of pass pp
    U4 dw;
    {
        const uint32_t kd = rg.kbase + (uint32_t)((l < P ? l : 0) * rows + row);
        dw = philox10((uint32_t)n, (uint32_t)(n >> 32), rg.dom(kd), (uint32_t)rg.oct(kd, s), g.seed);
    }
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
        const uint32_t ld = (uint32_t)(pp * rows + row);
        const bool valid = ld < rg.nvalid;
        Planes<H> pl;
        uint32_t m[13];
        compute_octant<H, false>(raw[pp], valid, l, sh.zbuf[row], pl, m);
        const uint32_t ux = bcast_lane(dw.x, pp), uy = bcast_lane(dw.y, pp), uz = bcast_lane(dw.z, pp);
        const int cs = row_class(sh.acc[ld], valid, unit53(ux, uy) * Rmax, l, row);
        select_site<H>(pl, cs, cs >= 0 ? sh.hist[ld][cs] : 0u, uz, l, &sh.selq[ld], g.st);
    }
    __syncthreads();
    long long F = 0, dM = 0, dB = 0;
    for (uint32_t t = tid; t < D; t += BLOCK) {
        const uint32_t f = sh.selq[t];
        if (t >= rg.nvalid || f == kNoEvent) continue;
        const uint32_t cs = f >> 12, q = f & 0xFFFu;
        flip_site<H>(g, rg.dom(rg.kbase + t), rg.oct(rg.kbase + t, s), q);
        F += 1;
        dM += cs >= 7 ? -2 : 2;              // the class carries the old spin
        dB += 12 - 4 * (long long)(cs % 7);  // and its aligned count
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
        for (int w = 0; w < BLOCK / 64; ++w) {
            F += sh.red[0][w];
            dM += sh.red[1][w];
            dB += sh.red[2][w];
        }
        if (F) atomicAdd((unsigned long long *)&g.st->acc_fired[0], (unsigned long long)F);
        if (dM) atomicAdd((unsigned long long *)&g.st->acc_dM[0], (unsigned long long)dM);
        if (dB) atomicAdd((unsigned long long *)&g.st->acc_dB[0], (unsigned long long)dB);
    }
}

// Many independent lattices in one launch: each workgroup finds its lattice by
// its workgroup index; lattices never wait for one another.
template <int H, int P, int BLOCK, bool INC>
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
    persistent_body<H, P, BLOCK, INC, 0>(R, blockIdx.x - R.first_wg, sh);  // lattices of either line count
}

// Before a launch: slots carry the generation of no cycle of this launch yet,
// flags the start cycle.
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
    uint32_t oct[kSlabDomains][kOctLds];    // active octants and their halos
    uint32_t sc[kSlabDomains][kSlabWords];  // slab counts of the active octants
    uint16_t cnt[kSlabDomains][8][14];      // class counts (the active octant; every octant for the all-octant R_max)
    double acc[kSlabDomains][14];           // running FP64 sums of the frequency lines
    double rk[kSlabDomains];
    uint32_t zbuf[kSlabRows][24];           // binning at launch start: z face words per row
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
// Spin at domain-local (x, y, z), each in [-2h, 4h), of the domain at c (the
// periodic neighbour domain outside [0, 2h)), and the domain, octant and local
// z of the site.
__device__ __forceinline__ uint32_t spin_at16(const Geom &g, DomainCoord c, int x, int y, int z, uint32_t &k,
                                              int &o, int &lz) {
    const int cx = x < 0 ? wrapm(c.kx, g.nd) : x >= 32 ? wrapp(c.kx, g.nd) : c.kx;
    const int cy = y < 0 ? wrapm(c.ky, g.nd) : y >= 32 ? wrapp(c.ky, g.nd) : c.ky;
    const int cz = z < 0 ? wrapm(c.kz, g.nd) : z >= 32 ? wrapp(c.kz, g.nd) : c.kz;
    x &= 31, y &= 31, z &= 31;
    o = (x >> 4) | ((y >> 4) << 1) | ((z >> 4) << 2);
    lz = z & 15;
    k = dindex(cx, cy, cz, g.nd);
    const uint32_t q = (uint32_t)((x & 15) + 16 * ((y & 15) + 16 * lz));
    const uint32_t word = (k * 8u + (uint32_t)o) * 128u + (q >> 5);
    return (ld32(&g.A[word]) >> (q & 31)) & 1u;
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
// site (its spin word and face copies) and moves its class; parts 1..3 move the
// classes of its two neighbours along axis part - 1.  A neighbour inside the
// octant takes its class from the octant and halo in LDS (o; the flipped site
// still reads its old spin there) and moves in the octant's counts in LDS (sc);
// one across a face reads its own neighbours from memory (none of them flips in
// the same cycle) and moves in that octant's counts by device atomics.  dco_k:
// the coordinates of domain k (kx | ky << 10 | kz << 20).
__device__ __forceinline__ void slab_flip_part(const Geom &g, const uint32_t *o, uint32_t *sc, uint32_t dco_k,
                                               uint32_t k, int so, uint32_t f, int part, long long &F,
                                               long long &dM, long long &dB) {
    const int cs = (int)(f >> 12);
    const uint32_t q = f & 0xFFFu;
    const int lx = (int)(q & 15u), ly = (int)((q >> 4) & 15u), lz = (int)(q >> 8);
    const uint32_t up = cs >= 7;
    if (part == 0) {
        slab_move_lds(sc, cs, site_class(!up, up ? cs - 7 : 6 - cs), lz >> 2);
        flip_site<16>(g, k, so, q);
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
    if (tid < 8) sh.rpred[tid] = 0.0;
    if (tid < 14) sh.r[tid] = g.r[tid];
    if (l < 8) sh.zbuf[row][16 + l] = 0;
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
    if (tid < 6) {
        uint32_t cnt = 0;
        for (uint32_t w = 0; w < G; ++w)
            if ((sh.nbr_bits[tid][w >> 5] >> (w & 31)) & 1u) {
                if (cnt < kMaxNbr) sh.nbr[tid][cnt] = w;
                ++cnt;
            }
        sh.nbr_cnt[tid] = cnt;
    }
    __syncthreads();

    // slab counts of all eight octants from the spins at launch start; they are
    // complete before this workgroup publishes its first R_max, hence before any
    // workgroup flips
#pragma unroll 1
    for (int o = 0; o < 8; ++o) slab_bin_octant(g, kbase, nvalid, o, sh);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    DevState *st = g.st;
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
                    if (!(l & 1)) {
                        o[kFxm + (l >> 1)] = raw[pp].xm;
                        o[kFxp + (l >> 1)] = raw[pp].xp;
                        o[kFym + (l >> 1)] = raw[pp].ym;
                        o[kFyp + (l >> 1)] = raw[pp].yp;
                    }
                    o[kFzm + l] = raw[pp].zw;  // lanes 8 .. 15: the face above
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
        // word and face copies) and its two neighbours along each axis.  A
        // neighbour inside the octant takes its class from the words in LDS (the
        // flipped site still reads its old spin there); one across a face reads
        // its own neighbours from memory (none of them flips in this cycle).
        {
            const uint32_t ld = (uint32_t)tid >> 2;
            const int part = tid & 3;
            const uint32_t f = ld < nvalid ? sh.selq[ld] : kNoEvent;
            if (f != kNoEvent)
                slab_flip_part(g, sh.oct[ld], sh.sc[ld], sh.dco[ld], kbase + ld, s, f, part, myF, mydM, mydB);
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
                    atomicAdd((unsigned long long *)&st->fired, (unsigned long long)F);
                    atomicAdd((unsigned long long *)&st->nulls,
                              (unsigned long long)((long long)nvalid * (long long)ncycles - F));
                    atomicAdd((unsigned long long *)&st->M, (unsigned long long)dM);
                    atomicAdd((unsigned long long *)&st->B, (unsigned long long)dB);
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
        if (tid < 64 && !sh.abort) {
            uint64_t start = now_ticks();
            for (uint32_t w = tid; w < G; w += 64)
                while (ld64(&xs.flag[w]) < n_end) {
                    __builtin_amdgcn_s_sleep(1);
                    if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                        atomicOr(&st->error, kErrFlagTimeout);
                        sh.abort = 1;
                        break;
                    }
                }
        }
        __syncthreads();
        if (tid < 64 && !sh.abort) {
            while (sh.pend_head != sh.pend_tail) {
                emit_record(g, xs, sh, G, tid, n0, fired0, nulls0, M0, B0);
                __builtin_amdgcn_wave_barrier();
            }
            if (tid == 0) {
                st->t = t;
                st->cycle = n_end;
                if (obs_every && (n_end % obs_every) == 0 && g.rec_cap) {
                    spkmc_record r;
                    r.cycle = n_end;
                    r.fired = ld64(&st->fired);
                    r.nulls = ld64(&st->nulls);
                    r.t = t;
                    r.M = (int64_t)ld64((const uint64_t *)&st->M);
                    r.B = (int64_t)ld64((const uint64_t *)&st->B);
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
    uint32_t oct[kSlabDomains][kOctLds];
    uint32_t sc[kSlabDomains][kSlabWords];
    double acc[kSlabDomains][14];
    uint32_t nbdom[kSlabDomains][6];
    uint32_t dco[kSlabDomains];
    uint32_t selq[kSlabDomains];
    uint32_t zbuf[kSlabRows][24];
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
    if (l < 8) sh.zbuf[row][16 + l] = 0;
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
        if (!(l & 1)) {
            oc[kFxm + (l >> 1)] = raw.xm;
            oc[kFxp + (l >> 1)] = raw.xp;
            oc[kFym + (l >> 1)] = raw.ym;
            oc[kFyp + (l >> 1)] = raw.yp;
        }
        oc[kFzm + l] = raw.zw;
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
            slab_flip_part(g, sh.oct[ld], sh.sc[ld], sh.dco[ld], rg.dom(rg.kbase + ld), rg.oct(rg.kbase + ld, s), f,
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
// Launch shapes.  A 16-lane row owns a domain; a workgroup runs `rows` rows
// and P passes (1, 2 or 4).  h = 16 keeps up to four passes of class planes in
// 256 registers with 32 rows (512 threads, two waves per SIMD); h = 8 needs 4
// registers per pass and runs 64 rows (1024 threads, four waves per SIMD).
int persist_rows(int h, bool) { return h == 8 ? 64 : 32; }
int persist_max_passes(int, bool) { return 4; }

template <int H, int P, int BLOCK>
static void *kernel_of(bool batch, bool inc, uint32_t lpd) {
    if (inc) return reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, true, 1>);
    if (batch) return reinterpret_cast<void *>(&k_persistent_batch<H, P, BLOCK, false>);
    return lpd == 4 ? reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 4>)
                    : reinterpret_cast<void *>(&k_persistent<H, P, BLOCK, false, 1>);
}
// Batches use the re-binning kernel (lines per domain read at run time).
static void *select_kernel(int h, int P, int block, bool batch = false, bool inc = false, uint32_t lpd = 1) {
    if (batch && inc) return nullptr;
    if (h == 16 && block == 512)
        return P == 1   ? kernel_of<16, 1, 512>(batch, inc, lpd)
               : P == 2 ? kernel_of<16, 2, 512>(batch, inc, lpd)
               : P == 4 ? kernel_of<16, 4, 512>(batch, inc, lpd)
                        : nullptr;
    if (h == 8 && block == 1024)
        return P == 1   ? kernel_of<8, 1, 1024>(batch, inc, lpd)
               : P == 2 ? kernel_of<8, 2, 1024>(batch, inc, lpd)
               : P == 4 ? kernel_of<8, 4, 1024>(batch, inc, lpd)
                        : nullptr;
    return nullptr;
}

bool persistent_supported(const Geom &g, const spkmc_params &p, bool inc, std::string &why) {
    if (g.layout != SPKMC_LAYOUT_PACKED) { why = "needs the PACKED layout"; return false; }
    if (g.h != 8 && g.h != 16) { why = "needs an octant edge of 8 or 16 (domain 16 or 32)"; return false; }
    // spins and face copies are read through buffer views with 32-bit byte offsets
    if (g.N / 8 >= (1ull << 31)) { why = "needs fewer than 2^34 sites"; return false; }
    const uint32_t ok = inc ? SPKMC_VARIANT_RMAX_ALL : (SPKMC_VARIANT_RMAX_BOUND | SPKMC_VARIANT_TWO_COLOURS);
    if (p.variant & ~ok) {
        why = inc ? "the incremental engine runs variants 0 and RMAX_ALL"
                  : "this engine runs variants 0, RMAX_BOUND and TWO_COLOURS";
        return false;
    }
    const int rows = persist_rows(g.h, inc), pmax = persist_max_passes(g.h, inc);
    const int pc = p.wg_domains / rows;
    if (p.wg_domains && (p.wg_domains % rows || pc > pmax || (pc & (pc - 1)))) {
        why = "wg_domains must be " + std::to_string(rows) + " times 1, 2" + (pmax == 4 ? " or 4" : "") +
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
    // the fewest passes whose workgroups are all resident at once (or the
    // requested domains per workgroup)
    for (int P = 1; P <= pmax; P <<= 1) {
        if (p.wg_domains && p.wg_domains != rows * P) continue;
        void *kern = select_kernel(g.h, P, block, false, inc, g.lpd);
        if (!kern) return hipErrorInvalidValue;
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, 0);
        if (e != hipSuccess) return e;
        const uint64_t D = (uint64_t)rows * P, G = ((uint64_t)g.K * g.lpd + D - 1) / D;
        if (occ > 0 && G <= (uint64_t)occ * cus && G <= (uint64_t)kMaxGrid) {
            grid = (int)G;
            wg_domains = (int)D;
            return hipSuccess;
        }
    }
    return hipErrorCooperativeLaunchTooLarge;
}

bool rows_supported(const Geom &g) {
    return g.layout == SPKMC_LAYOUT_PACKED && (g.h == 8 || g.h == 16) && !(g.variant & SPKMC_VARIANT_RMAX_ALL) &&
           g.N / 8 < (1ull << 31);
}

template <int H, int BLOCK, int P>
static hipError_t launch_rows(const Geom &g, uint64_t n, hipStream_t stream) {
    const uint64_t lines = (uint64_t)g.K * g.lpd;
    constexpr uint32_t D = RowsGeometry<H, BLOCK, 1, P>::D;
    const uint32_t grid = (uint32_t)((lines + D - 1) / D);
    if (g.lpd == 4) {
        hipLaunchKernelGGL((k_rows_bin<H, BLOCK, 4, P>), dim3(grid), dim3(BLOCK), 0, stream, g, n);
        hipLaunchKernelGGL((k_rows_select<H, BLOCK, 4, P>), dim3(grid), dim3(BLOCK), 0, stream, g, n);
    } else {
        hipLaunchKernelGGL((k_rows_bin<H, BLOCK, 1, P>), dim3(grid), dim3(BLOCK), 0, stream, g, n);
        hipLaunchKernelGGL((k_rows_select<H, BLOCK, 1, P>), dim3(grid), dim3(BLOCK), 0, stream, g, n);
    }
    return hipGetLastError();
}

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

hipError_t launch_cycle_rows(const Geom &g, uint64_t n, hipStream_t stream) {
    if (!rows_supported(g)) return hipErrorInvalidValue;
    return g.h == 16 ? launch_rows<16, 512, kRowsPasses>(g, n, stream) : launch_rows<8, 1024, kRowsPasses>(g, n, stream);
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

uint64_t persistent_scratch_words(uint64_t K) { return kScratchWordsPerWg * (K / 16 + 2) + 16; }

PersistScratch scratch_of(const Geom &g, int G) {
    PersistScratch xs;
    xs.slot = g.sync;
    xs.flag = g.sync + 2 * (uint64_t)G;
    xs.recp = reinterpret_cast<int64_t *>(g.sync + 3 * (uint64_t)G);
    xs.emitted = g.sync + 15 * (uint64_t)G;  // within the 16 spare words
    return xs;
}

hipError_t launch_persistent(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid, int block,
                             int wg_domains, bool inc, hipStream_t stream) {
    PersistScratch xs = scratch_of(g, grid);
    int P = wg_domains / (block / 16);
    void *kern = select_kernel(g.h, P, block, false, inc, g.lpd);
    if (!kern) return hipErrorInvalidValue;
    const uint64_t ndh = inc ? (uint64_t)g.K * 16 : 0;
    uint64_t blocks = ((uint64_t)grid + 255) / 256, bdh = (ndh + 255) / 256;
    blocks = blocks > bdh ? blocks : (bdh < 2048 ? bdh : 2048);
    hipLaunchKernelGGL(k_persistent_prep, dim3((uint32_t)blocks), dim3(256), 0, stream, xs, (uint32_t)grid, n0, g.dh, ndh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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

hipError_t launch_slab(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid,
                       hipStream_t stream) {
    if (!g.sc || g.h != 16) return hipErrorInvalidValue;
    PersistScratch xs = scratch_of(g, grid);
    hipLaunchKernelGGL(k_persistent_prep, dim3((uint32_t)((grid + 255) / 256)), dim3(256), 0, stream, xs,
                       (uint32_t)grid, n0, g.dh, (uint64_t)0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
    return hipLaunchCooperativeKernel(slab_kernel(g), dim3(grid), dim3(kSlabBlock), args, 0,
                                      stream);
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
uint32_t batch_capacity(int h, int P) {
    const int block = persist_rows(h, false) * 16;
    void *kern = select_kernel(h, P, block, true);
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
                      uint32_t n, int P, Replica *out, int &grid, int &block) {
    if (n == 0) return hipErrorInvalidValue;
    const int h = gs[0]->h;
    block = persist_rows(h, false) * 16;
    void *kern = select_kernel(h, P, block, true);
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
    const uint32_t cap = batch_capacity(h, P);
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

// After a captured macro-step: every lattice's next replay starts where this
// one stopped.
__global__ void k_advance_batch(Replica *reps, uint32_t nrep) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrep) reps[i].n0 += reps[i].ncycles;
}

// The descriptors must already be in device memory (dev_reps).
hipError_t launch_batch(const Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, hipStream_t stream) {
    void *kern = select_kernel(h, P, block, true);
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
hipError_t capture_batch(Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, hipGraph_t *graph) {
    void *kern = select_kernel(h, P, block, true);
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
