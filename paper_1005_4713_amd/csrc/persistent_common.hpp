// persistent_common.hpp -- device code shared by the kernel files of the gfx950
// spkMC library (kernels_persistent.hip, kernels_rows.hip, kernels_slab.hip):
// launch-wide constants and descriptors, buffer views, v_bitop3 / DPP helpers,
// the bit-sliced class planes of an octant (loads, neighbours, 6-input count,
// popcount moments), the histogram from the moments, row scans and maxima, the
// selection of a row's class and site, the flip of a site with the halo copies it is in,
// the bounded neighbour waits and the record sums of the persistent launches.
#pragma once

#include "spkmc_device.hpp"

namespace spkmc {

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
    int64_t *fin;       // G x 3: each workgroup's totals (fired, dM, dB) at the end of the launch
    uint64_t *emitted;  // records of this launch appended so far (fixed-bound variant); 0 between launches
    double *rpred;      // 8: the last R_max of each colour, the next launch's first predictions
};
constexpr uint64_t kScratchWordsPerWg = 2 + 1 + 3 * kRecBanks + 3;

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
// Buffer views of the packed spins and of the halo copies (byte offsets below
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
__device__ __forceinline__ uint32_t ld_face(const Views &v, bool valid, uint32_t w) {  // word w of the halo copies
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

// The six halo faces of octant (k, s): the layers of the octants of colour
// s ^ (1 << axis) that touch it from below (their layer at local coordinate
// h - 1) and from above (layer 0), kept by every octant as its own copy in F
// (halo slots x below, x above, y below, y above, z below, z above; flips push
// into them), so that an octant's halo is one contiguous 6 h^2 / 8 bytes.
struct HaloFaces {
    uint32_t lo[3];  // word index in F of the halo face below along each axis
    uint32_t hi[3];  // word index in F of the halo face above
};
// (32-bit word indices from the uniform base: F holds K * 48 h^2 / 32 words,
// below 2^31 for every supported size)
template <int H>
__device__ __forceinline__ HaloFaces halo_faces(uint32_t k, int s, const uint32_t *) {
    HaloFaces hf;
    constexpr uint32_t fw = H * H / 32, fwpo = 6 * fw;  // words per face, per octant
    // domain indices stay below 2^22 (fewer than 2^34 sites, at least 4096 per
    // domain): a 24-bit multiply
    const uint32_t base = __umul24(k, 8u * fwpo) + (uint32_t)s * fwpo;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        hf.lo[a] = base + (uint32_t)(2 * a) * fw;
        hf.hi[a] = base + (uint32_t)(2 * a + 1) * fw;
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
    uint32_t W[8];  // own plane: word p = rows 2p, 2p + 1
    // the octant's six halo faces (8 words each: x below, x above, y below, y
    // above, z below, z above), a quarter-face per lane: lane j < 12 holds words
    // 4 (j & 1) .. 4 (j & 1) + 3 of face j / 2; lanes 12 .. 15 hold zeros
    uint32_t F[4];
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
// The six halo faces: one 16-byte device-coherent load per lane (a halo face is
// 8 words at a 32-byte aligned address).
__device__ __forceinline__ void load16_faces(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                             Raw<16> &r) {
    const HaloFaces hf = halo_faces<16>(k, s, nb);
    const Views vw = views_of(g);
    // face f = l / 2 (selects, not an indexed read: the faces stay in registers)
    const int f = l >> 1;
    uint32_t base = hf.lo[0];
    base = f == 1 ? hf.hi[0] : base;
    base = f == 2 ? hf.lo[1] : base;
    base = f == 3 ? hf.hi[1] : base;
    base = f == 4 ? hf.lo[2] : base;
    base = f == 5 ? hf.hi[2] : base;
    const int off = valid && l < 12 ? (int)((base + 4u * (uint32_t)(l & 1)) * 4u) : vw.endF;
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(vw.F, off, 0, kCoherent);
    r.F[0] = v[0];
    r.F[1] = v[1];
    r.F[2] = v[2];
    r.F[3] = v[3];
}

// zrow: this row's kRowHalo LDS words: the six halo faces (8 words each, in the
// order of Raw<16>::F), then 8 zeros.
constexpr int kRowHalo = 56;
// MOM: also accumulate the 13 popcount moments of the octant.
template <bool MOM>
__device__ __forceinline__ void compute16(const Raw<16> &r, bool valid, int l, uint32_t *zrow, Planes<16> &P,
                                          uint32_t (&m)[13]) {
    // the faces into the row's LDS words; the row's own lanes read them back (same wavefront)
    if (l < 12) *reinterpret_cast<uint4 *>(zrow + 4 * l) = uint4{r.F[0], r.F[1], r.F[2], r.F[3]};
    // the reads below take words other lanes wrote: no reordering across this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t *zlo = zrow + (l == 0 ? 32 : 48), *zhi = zrow + (l == 15 ? 40 : 48);
    // x faces: bit ly + 16 lz -> half-word l of the face; y faces: bit lx + 16 lz -> half-word l
    const uint32_t sh16 = 16 * (l & 1);
    const uint32_t xm = (zrow[l >> 1] >> sh16) & 0xFFFFu, xp = (zrow[8 + (l >> 1)] >> sh16) & 0xFFFFu;
    const uint32_t ym = (zrow[16 + (l >> 1)] >> sh16) & 0xFFFFu, yp = (zrow[24 + (l >> 1)] >> sh16) & 0xFFFFu;
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
                                           Raw<H> &r) {
    if constexpr (H == 16) load16_faces(g, k, s, valid, l, nb, r);
    else load8_faces(g, k, s, valid, l, nb, 7, r);
}
template <int H>
__device__ __forceinline__ void load_octant(const Geom &g, uint32_t k, int s, bool valid, int l, const uint32_t *nb,
                                            Raw<H> &r) {
    load_words<H>(g, k, s, valid, l, r);
    load_faces<H>(g, k, s, valid, l, nb, r);
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

// Sum over each group of four lanes of a DPP row, in the group's last lane (lane
// 4j + 3 ends with lanes 4j .. 4j + 3): two shifted adds.
__device__ __forceinline__ uint32_t quad_sum(uint32_t v) {
    v += dpp0<kRowShr1>(v);
    v += dpp0<kRowShr2>(v);
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
        uint32_t wsel = 0, before = 0, msk = mk[0];
        if constexpr (WPL == 8) {
            // the first word whose running count exceeds r0, by halving (the
            // running counts never decrease)
            const bool c1 = cum[3] <= r0;
            const uint32_t a0 = c1 ? cum[4] : cum[0], a1 = c1 ? cum[5] : cum[1], a2 = c1 ? cum[6] : cum[2];
            const uint32_t m0 = c1 ? mk[4] : mk[0], m1 = c1 ? mk[5] : mk[1], m2 = c1 ? mk[6] : mk[2],
                           m3 = c1 ? mk[7] : mk[3];
            before = c1 ? cum[3] : 0u;
            const bool c2 = a1 <= r0;
            const uint32_t x0 = c2 ? a2 : a0, n0 = c2 ? m2 : m0, n1 = c2 ? m3 : m1;
            before = c2 ? a1 : before;
            const bool c3 = x0 <= r0;
            msk = c3 ? n1 : n0;
            before = c3 ? x0 : before;
            wsel = (c1 ? 4u : 0u) | (c2 ? 2u : 0u) | (c3 ? 1u : 0u);
        } else {
#pragma unroll
            for (int p = 0; p + 1 < WPL; ++p) wsel += cum[p] <= r0 ? 1u : 0u;
#pragma unroll
            for (int p = 1; p < WPL; ++p)
                if (wsel == (uint32_t)p) {
                    before = cum[p - 1];
                    msk = mk[p];
                }
        }
        const uint32_t q = (uint32_t)(l * WPL) * 32 + wsel * 32 + (uint32_t)nth_set_bit(msk, r0 - before);
        *slot = ((uint32_t)cs << 12) | q;  // after lane 0's store, same wavefront
    }
}

// Flip site q of octant (k, so): its spin word, and the halo copy of every
// octant whose halo it is in (the octant across each of its octant's boundary
// layers it lies on).  nb holds the six neighbour domains of k (-x, +x, -y,
// +y, -z, +z).
template <int H>
__device__ __forceinline__ void flip_site(const Geom &g, uint32_t k, int so, uint32_t q, const uint32_t *nb) {
    // 32-bit word indices: fewer than 2^34 sites (the spins' and the copies' words below 2^31)
    constexpr uint32_t wpo = H * H * H / 32, fwpo = 6 * H * H / 32;
    flip_word(g.A + ((k * 8u + (uint32_t)so) * wpo + (q >> 5)), 1u << (q & 31));
    const uint32_t c[3] = {q % H, (q / H) % H, q / (H * H)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (c[a] != 0 && c[a] != H - 1) continue;
        // the site's place in a face: the other two coordinates, the lower axis first
        const uint32_t u = a == 0 ? c[1] : c[0], v = a == 2 ? c[1] : c[2];
        const uint32_t bit = u + H * v;
        const bool below = c[a] == 0;  // layer 0: the halo above of the octant below
        const bool inner = (((so >> a) & 1) != 0) == below;  // the octant across is in this domain
        const uint32_t kt = inner ? k : nb[2 * a + (below ? 0 : 1)];
        const uint32_t ot = (uint32_t)(so ^ (1 << a));
        const uint32_t slot = (uint32_t)(2 * a + (below ? 1 : 0));
        const uint32_t b = slot * H * H + bit;
        flip_word(g.F + ((kt * 8u + ot) * fwpo + (b >> 5)), 1u << (b & 31));
    }
}

// wall clock (100 MHz) for bounded waits
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

}  // namespace

// Sums and waits over the workgroups of a launch at its end, one wavefront: lane
// i takes workgroups i, i + 64, ...  Each lane's loads for kWgPerLane workgroups
// go out together, so 256 workgroups cost one round trip (not one per load).
constexpr int kWgPerLane = 4;

// The (fired, dM, dB) triples p[3w .. 3w + 2] of workgroups w < G, summed over
// the wavefront (every lane ends with the totals).
__device__ __forceinline__ void sum_triples(const int64_t *p, uint32_t G, int lane, long long &F, long long &dM,
                                            long long &dB) {
    F = dM = dB = 0;
    for (uint32_t base = 0; base < G; base += 64 * kWgPerLane) {
        uint64_t v[kWgPerLane][3];
#pragma unroll
        for (int i = 0; i < kWgPerLane; ++i) {
            const uint32_t w = base + (uint32_t)(i * 64 + lane);
            const uint32_t wc = w < G ? w : G - 1;  // lanes past the end read a valid word and drop it
#pragma unroll
            for (int j = 0; j < 3; ++j) v[i][j] = ld64(reinterpret_cast<const uint64_t *>(&p[3 * wc + j]));
        }
#pragma unroll
        for (int i = 0; i < kWgPerLane; ++i)
            if (base + (uint32_t)(i * 64 + lane) < G) {
                F += (long long)v[i][0];
                dM += (long long)v[i][1];
                dB += (long long)v[i][2];
            }
    }
    for (int o = 32; o > 0; o >>= 1) {
        F += __shfl_xor(F, o);
        dM += __shfl_xor(dM, o);
        dB += __shfl_xor(dB, o);
    }
}

// Wait (one wavefront) until every workgroup's flag has reached `upto`; only
// the flags not yet there are read again.  false on a timeout or a device
// error (error set, sh.abort raised).
template <class SH>
__device__ __forceinline__ bool wait_all_flags(const PersistScratch &xs, DevState *st, SH &sh, uint32_t G,
                                               int lane, uint64_t upto) {
    const uint64_t start = now_ticks();
    for (uint32_t base = 0; base < G; base += 64 * kWgPerLane) {
        uint64_t fv[kWgPerLane];
#pragma unroll
        for (int i = 0; i < kWgPerLane; ++i) {
            const uint32_t w = base + (uint32_t)(i * 64 + lane);
            fv[i] = w < G ? ld64(&xs.flag[w]) : upto;
        }
        for (;;) {
            bool done = true;
#pragma unroll
            for (int i = 0; i < kWgPerLane; ++i)
                if (fv[i] < upto) {
                    done = false;
                    fv[i] = ld64(&xs.flag[base + (uint32_t)(i * 64 + lane)]);
                }
            if (__all(done)) break;
            __builtin_amdgcn_s_sleep(1);
            if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                atomicOr(&st->error, kErrFlagTimeout);
                sh.abort = 1;
                return false;
            }
        }
    }
    return true;
}

// Sum the partials of the oldest pending record over all workgroups (one
// wavefront) and append the record.  The caller guarantees every workgroup has
// stored them.  (A lane's loads are not batched here as in sum_triples: inside
// the main loop that code slowed the cycle of the batch kernels by a tenth and
// the single-lattice cycle by 1 %, even in launches that emit no record.)
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
    // the directions' lists laid end to end, one flag per thread: every thread
    // waits on its own flag, so all directions cost one round trip together
    const int d0 = dir < 0 ? 0 : dir, d1 = dir < 0 ? 6 : dir + 1;
    uint32_t total = 0;
    for (int d = d0; d < d1; ++d) total += sh.nbr_cnt[d] > kMaxNbr ? G : sh.nbr_cnt[d];
    for (uint32_t j = tid; j < total; j += BLOCK) {
        uint32_t i = j;
        int d = d0;
        for (;;) {
            const uint32_t cnt = sh.nbr_cnt[d] > kMaxNbr ? G : sh.nbr_cnt[d];
            if (i < cnt) break;
            i -= cnt;
            ++d;
        }
        const uint32_t w = sh.nbr_cnt[d] > kMaxNbr ? i : sh.nbr[d][i];
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
    __syncthreads();
    return !sh.abort;
}

// The lines of a row-kernel workgroup (the per-cycle row and slab kernels).
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

// The sync scratch of a persistent launch of G workgroups (kernels_persistent.hip),
// and its set-up before a launch starting at cycle n0.
PersistScratch scratch_of(const Geom &g, int G);
hipError_t launch_persistent_prep(const PersistScratch &xs, uint32_t G, uint64_t n0, hipStream_t stream);

// The neighbour workgroups of this workgroup per direction, from the bitmap
// sh.nbr_bits (one thread per direction, a word of the bitmap at a time).
template <class SH>
__device__ __forceinline__ void list_neighbours(SH &sh, uint32_t G) {
    const int d = threadIdx.x;
    if (d < 6) {
        uint32_t cnt = 0;
        for (uint32_t wd = 0; wd < (G + 31) / 32; ++wd) {
            uint32_t bits = sh.nbr_bits[d][wd];
            while (bits) {
                const uint32_t w = wd * 32 + (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1;
                if (cnt < kMaxNbr) sh.nbr[d][cnt] = w;
                ++cnt;
            }
        }
        sh.nbr_cnt[d] = cnt;
    }
}

// The first predictions of a launch: the last R_max of each colour left by the
// previous launch of the lattice (0 = none; a prediction only decides which
// selection is tried first, never the outcome).
template <class SH>
__device__ __forceinline__ void load_predictions(SH &sh, const PersistScratch &xs) {
    const int c = threadIdx.x;
    if (c < 8) {
        const double v = xs.rpred[c];
        sh.rpred[c] = (v > 0.0 && v < 1.0e300) ? v : 0.0;
    }
}

// End of a launch in every workgroup: its totals since launch start into its
// own words (read by the recorder once every flag has reached the last cycle).
__device__ __forceinline__ void store_final(const PersistScratch &xs, uint32_t gid, long long F, long long dM,
                                            long long dB) {
    st64(reinterpret_cast<uint64_t *>(&xs.fin[3 * gid]), (uint64_t)F);
    st64(reinterpret_cast<uint64_t *>(&xs.fin[3 * gid + 1]), (uint64_t)dM);
    st64(reinterpret_cast<uint64_t *>(&xs.fin[3 * gid + 2]), (uint64_t)dB);
}

// The recorder (one wavefront) after every workgroup has finished: the totals
// of the launch folded into the lattice's counters (NLc = frequency lines times
// cycles of the launch), the predictions kept for the next launch, and the
// fixed-bound record counter reset.
template <class SH>
__device__ __forceinline__ void fold_final(const Geom &g, const PersistScratch &xs, SH &sh, uint32_t G, int lane,
                                           uint64_t NLc, uint64_t fired0, uint64_t nulls0, int64_t M0, int64_t B0) {
    long long F, dM, dB;
    sum_triples(xs.fin, G, lane, F, dM, dB);
    if (lane < 8) xs.rpred[lane] = sh.rpred[lane];
    if (lane == 0) {
        DevState *st = g.st;
        st->fired = fired0 + (uint64_t)F;
        st->nulls = nulls0 + NLc - (uint64_t)F;
        st->M = M0 + dM;
        st->B = B0 + dB;
        *xs.emitted = 0;
    }
}

}  // namespace spkmc
