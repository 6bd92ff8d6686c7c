// kernels_persistent.hip -- the persistent ("PERSISTENT") engine of the gfx950
// spkMC library: one cooperative launch runs many cycles (Sec. 3.1 steps 1-6
// with the sublattice steps 4a/4b of Sec. 3.2) over a bit-packed lattice.
//
// Work decomposition
//   * A 16-lane DPP row owns one domain; a workgroup of B threads owns
//     D = P * B / 16 consecutive domains (numbered kx + nd (ky + nd kz)) for the
//     whole launch, processed in P passes whose per-site state stays in
//     registers across the R_max exchange.
//   * h = 16: lane l of the row holds plane lz = l of the octant (8 words, two
//     16-site x rows each); h = 8: lane l holds word l (four 8-site rows of
//     plane l / 2).  The z neighbours come from the adjacent lanes through DPP
//     row shifts, the y neighbours from the word below / above, the x
//     neighbours from in-word shifts; the 1-site halo comes from the face
//     copies of the six neighbouring octants.
//   * The number of up neighbours of 32 sites is counted bit-sliced (two full
//     adders and a 2-bit add), and the 14-class histogram of the octant is
//     recovered from 13 popcounts of products of the count bit planes and the
//     spin plane (inclusion-exclusion; n_up = 7 never occurs).
//
// Synchronisation (no cache-flushing fences: every word another workgroup may
// write is read with device-coherent loads, and every write is an atomic)
//   * R_max (step 2): each workgroup stores its local maximum with the cycle
//     parity in the sign bit (all rates are positive) into its own slot and
//     polls all slots; the maximum is exact and order-free.
//   * boundary events (step 6): after its flips a workgroup publishes the
//     cycle number in its flag.  Before binning cycle n + 1 a workgroup only
//     waits for the neighbouring workgroups the colour change s_n -> s_n+1
//     makes it depend on: the halo of colour s' holds flipped sites of colour
//     s_n only if s_n = s' ^ (1 << b), and then only from the neighbour domain
//     along axis b.
//   * the clock (step 5) is advanced identically by every workgroup;
//     counters are reduced at observation cycles and at the end of the launch.
// Every wait is bounded in wall-clock time; a timeout sets DevState::error and
// every workgroup leaves the loop.
#include <string>

#include "spkmc_device.hpp"

namespace spkmc {

namespace {

constexpr int kMaxNbr = 16;           // neighbour workgroups per direction kept in LDS
constexpr int kMaxGrid = 2048;        // workgroups of one persistent launch
constexpr uint64_t kTimeoutTicks = 200000000ull;  // 2 s of the 100 MHz wall clock

// Device scratch of the persistent engine (its own region of the state, 9 G words).
struct PersistScratch {
    uint64_t *slot;     // 2 x G: R_max of each workgroup; bank n & 1, generation (n >> 1) & 1 in bit 63
    uint64_t *flag;     // G: cycles whose flips are complete
    int64_t *recp;      // 2 x G x 3: record partials (fired, dM, dB) since launch start
};

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
__device__ __forceinline__ uint32_t flip_word(uint32_t *p, uint32_t m) {
    return __hip_atomic_fetch_xor(p, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, 0xF, false);
}
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114,
              kRowShr8 = 0x118;

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
// above (x0/y0/z0 face).
struct HaloFaces {
    const uint32_t *lo[3];  // face at local coordinate h - 1 of the octant below
    const uint32_t *hi[3];  // face at local coordinate 0 of the octant above
};
__device__ __forceinline__ HaloFaces halo_faces(const Geom &g, uint32_t k, int s) {
    DomainCoord c = dcoord(k, g.nd);
    int kc[3] = {c.kx, c.ky, c.kz};
    HaloFaces hf;
    const uint32_t fw = g.h2 / 32;  // words per face
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int bit = (s >> a) & 1;
        int nb = s ^ (1 << a);
        int km[3] = {kc[0], kc[1], kc[2]}, kp[3] = {kc[0], kc[1], kc[2]};
        if (!bit) km[a] = wrapm(kc[a], g.nd);  // below lies in the previous domain
        if (bit) kp[a] = wrapp(kc[a], g.nd);   // above lies in the next domain
        uint32_t kmi = dindex(km[0], km[1], km[2], g.nd), kpi = dindex(kp[0], kp[1], kp[2], g.nd);
        hf.lo[a] = g.F + ((uint64_t)kmi * 8 + nb) * g.fwpo + (2 * a + 1) * fw;
        hf.hi[a] = g.F + ((uint64_t)kpi * 8 + nb) * g.fwpo + (2 * a) * fw;
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

__device__ __forceinline__ void count6(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f,
                                       uint32_t &o0, uint32_t &o1, uint32_t &o2) {
    uint32_t s1 = a ^ b ^ c, c1 = (a & b) | (c & (a ^ b));
    uint32_t s2 = d ^ e ^ f, c2 = (d & e) | (f & (d ^ e));
    o0 = s1 ^ s2;
    uint32_t k0 = s1 & s2;
    o1 = c1 ^ c2 ^ k0;
    o2 = (c1 & c2) | (k0 & (c1 ^ c2));
}

// 13 moments: pop(S), pop(b0), pop(b1), pop(b2), pop(b0b1), pop(b0b2), pop(b1b2)
// and the same six products with S.
__device__ __forceinline__ void moments(uint32_t S, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t (&m)[13]) {
    uint32_t p01 = b0 & b1, p02 = b0 & b2, p12 = b1 & b2;
    m[0] += __builtin_popcount(S);
    m[1] += __builtin_popcount(b0);
    m[2] += __builtin_popcount(b1);
    m[3] += __builtin_popcount(b2);
    m[4] += __builtin_popcount(p01);
    m[5] += __builtin_popcount(p02);
    m[6] += __builtin_popcount(p12);
    m[7] += __builtin_popcount(S & b0);
    m[8] += __builtin_popcount(S & b1);
    m[9] += __builtin_popcount(S & b2);
    m[10] += __builtin_popcount(S & p01);
    m[11] += __builtin_popcount(S & p02);
    m[12] += __builtin_popcount(S & p12);
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

// --- h = 16 --------------------------------------------------------------------
// lane l = plane lz; word p holds rows ly = 2p (bits 0..15) and 2p + 1 (bits 16..31).
__device__ __forceinline__ void bin_octant16(const Geom &g, uint32_t k, int s, bool valid, int l,
                                             Planes<16> &P, uint32_t (&m)[13]) {
    uint32_t W[8], zf[8];
    uint32_t xm = 0, xp = 0, ym = 0, yp = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) { W[p] = 0; zf[p] = 0; }
    if (valid) {
        const uint32_t *A = g.A + ((uint64_t)k * 8 + s) * 128 + l * 8;
#pragma unroll
        for (int p = 0; p < 8; p += 2) {
            uint64_t v = ld_words2(A + p);
            W[p] = (uint32_t)v;
            W[p + 1] = (uint32_t)(v >> 32);
        }
        HaloFaces hf = halo_faces(g, k, s);
        // x faces: bit ly + 16 lz -> half-word l; y faces: bit lx + 16 lz -> half-word l
        xm = (ld32(hf.lo[0] + (l >> 1)) >> (16 * (l & 1))) & 0xFFFFu;
        xp = (ld32(hf.hi[0] + (l >> 1)) >> (16 * (l & 1))) & 0xFFFFu;
        ym = (ld32(hf.lo[1] + (l >> 1)) >> (16 * (l & 1))) & 0xFFFFu;
        yp = (ld32(hf.hi[1] + (l >> 1)) >> (16 * (l & 1))) & 0xFFFFu;
        // z faces (bit lx + 16 ly, the layout of a plane): plane 0 needs the face
        // below, plane 15 the face above; the DPP shifts keep them in those lanes
        if (l == 0 || l == 15) {
            const uint32_t *zface = l == 0 ? hf.lo[2] : hf.hi[2];
#pragma unroll
            for (int p = 0; p < 8; p += 2) {
                uint64_t v = ld_words2(zface + p);
                zf[p] = (uint32_t)v;
                zf[p + 1] = (uint32_t)(v >> 32);
            }
        }
    }
    // x halo bits: for word p, bit 0 <- xm bit 2p, bit 16 <- xm bit 2p+1 (and bits 15, 31 for xp)
    uint32_t Tm = xm | (xm << 15), Tp = xp | (xp << 15);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        uint32_t w = W[p];
        uint32_t nxm = ((w << 1) & 0xFFFEFFFEu) | ((Tm >> (2 * p)) & 0x00010001u);
        uint32_t nxp = ((w >> 1) & 0x7FFF7FFFu) | (((Tp >> (2 * p)) & 0x00010001u) << 15);
        uint32_t nym = p == 0 ? ((w << 16) | ym) : align_hi(w, W[p - 1], 16);
        uint32_t nyp = p == 7 ? ((yp << 16) | (w >> 16)) : align_hi(W[p + 1], w, 16);
        uint32_t nzm = dpp<kRowShr1>(zf[p], w);  // plane lz - 1, or the face below at lz = 0
        uint32_t nzp = dpp<kRowShl1>(zf[p], w);  // plane lz + 1, or the face above at lz = 15
        uint32_t o0, o1, o2;
        count6(nxm, nxp, nym, nyp, nzm, nzp, o0, o1, o2);
        P.S[p] = w;
        P.b0[p] = o0;
        P.b1[p] = o1;
        P.b2[p] = o2;
        if (valid) moments(w, o0, o1, o2, m);
    }
}

// --- h = 8 ---------------------------------------------------------------------
// lane l = 2 lz + p holds word l: rows ly = 4p .. 4p + 3 of plane lz, 8 bits each.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) {  // bits 0..3 -> bits 0, 8, 16, 24
    return (nib * 0x00204081u) & 0x01010101u;
}
__device__ __forceinline__ void bin_octant8(const Geom &g, uint32_t k, int s, bool valid, int l, Planes<8> &P,
                                            uint32_t (&m)[13]) {
    int lz = l >> 1, p = l & 1;
    uint32_t w = 0, xm = 0, xp = 0, yface = 0, zface = 0;
    if (valid) {
        w = ld32(g.A + ((uint64_t)k * 8 + s) * 16 + l);
        HaloFaces hf = halo_faces(g, k, s);
        // x faces: bit ly + 8 lz; rows 4p..4p+3 of plane lz = bits 4l .. 4l + 3
        xm = (ld32(hf.lo[0] + (l >> 3)) >> (4 * (l & 7))) & 0xFu;
        xp = (ld32(hf.hi[0] + (l >> 3)) >> (4 * (l & 7))) & 0xFu;
        // y faces: bit lx + 8 lz = byte lz; the lowest row of p = 0 needs the face below,
        // the highest row of p = 1 the face above
        const uint32_t *yf = p == 0 ? hf.lo[1] : hf.hi[1];
        yface = (ld32(yf + (lz >> 2)) >> (8 * (lz & 3))) & 0xFFu;
        // z faces: bit lx + 8 ly, word p covers rows 4p .. 4p + 3
        if (lz == 0) zface = ld32(hf.lo[2] + p);
        if (lz == 7) zface = ld32(hf.hi[2] + p);
    }
    uint32_t nxm = ((w << 1) & 0xFEFEFEFEu) | spread4(xm);
    uint32_t nxp = ((w >> 1) & 0x7F7F7F7Fu) | (spread4(xp) << 7);
    uint32_t below = dpp<kRowShr1>(0u, w);  // word l - 1 (row 4p - 1 when p = 1)
    uint32_t above = dpp<kRowShl1>(0u, w);  // word l + 1 (row 4p + 4 when p = 0)
    uint32_t nym = p ? align_hi(w, below, 24) : ((w << 8) | yface);
    uint32_t nyp = p ? ((yface << 24) | (w >> 8)) : align_hi(above, w, 8);
    uint32_t nzm = dpp<kRowShr2>(zface, w);  // plane lz - 1 (lanes 0, 1 keep the face below)
    uint32_t nzp = dpp<kRowShl2>(zface, w);  // plane lz + 1 (lanes 14, 15 keep the face above)
    uint32_t o0, o1, o2;
    count6(nxm, nxp, nym, nyp, nzm, nzp, o0, o1, o2);
    P.S[0] = w;
    P.b0[0] = o0;
    P.b1[0] = o1;
    P.b2[0] = o2;
    if (valid) moments(w, o0, o1, o2, m);
}

template <int H>
__device__ __forceinline__ void bin_octant(const Geom &g, uint32_t k, int s, bool valid, int l, Planes<H> &P,
                                           uint32_t (&m)[13]) {
    if constexpr (H == 16) bin_octant16(g, k, s, valid, l, P, m);
    else bin_octant8(g, k, s, valid, l, P, m);
}

// Inclusive prefix sum over the 16 lanes of a DPP row (lane 15 ends with the
// row total): four shifted adds, lanes shifted in from outside the row add 0.
__device__ __forceinline__ uint32_t row_scan(uint32_t v) {
    v += dpp<kRowShr1>(0u, v);
    v += dpp<kRowShr2>(0u, v);
    v += dpp<kRowShr4>(0u, v);
    v += dpp<kRowShr8>(0u, v);
    return v;
}

// wall clock (100 MHz) for bounded waits
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

}  // namespace

// Workgroup-shared state of the persistent kernel.
constexpr int kMaxWgDomains = 256;
struct PersistShared {
    double r[14];                       // rate table
    uint32_t mom[kMaxWgDomains][13];    // per domain: the 13 popcount moments of its active octant
    uint32_t hist[kMaxWgDomains][14];   // per domain: class histogram
    double acc[kMaxWgDomains][14];      // per domain: running FP64 sums of the frequency line
    double rk[kMaxWgDomains];
    double rmax;
    int abort;
    uint32_t nbr_bits[6][kMaxGrid / 32];  // neighbour workgroups per direction, as a bitmap
    uint32_t nbr_cnt[6];                  // > kMaxNbr: too many, wait for every workgroup
    uint32_t nbr[6][kMaxNbr];
    long long red[3][16];
};

template <int H, int P, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_persistent(Geom g, PersistScratch xs, uint64_t n0, uint64_t ncycles,
                                                     uint32_t obs_every) {
    __shared__ PersistShared sh;
    const int tid = threadIdx.x;
    const int nthr = BLOCK;
    const int rows = nthr >> 4;              // domains per pass
    const int row = tid >> 4, l = tid & 15;  // DPP row and lane inside it
    const uint32_t G = gridDim.x, gid = blockIdx.x;
    const uint32_t D = (uint32_t)(rows * P);
    const uint32_t kbase = gid * D;
    const uint32_t nvalid = kbase >= g.K ? 0u : (g.K - kbase < D ? g.K - kbase : D);

    // neighbour workgroups per direction (0: -x, 1: +x, 2: -y, 3: +y, 4: -z, 5: +z)
    for (uint32_t i = tid; i < 6 * (kMaxGrid / 32); i += nthr) (&sh.nbr_bits[0][0])[i] = 0;
    if (tid == 0) sh.abort = 0;
    if (tid < 14) sh.r[tid] = g.r[tid];
    __syncthreads();
    for (uint32_t i = tid; i < nvalid * 6; i += nthr) {
        uint32_t k = kbase + i / 6;
        int dir = (int)(i % 6), a = dir >> 1;
        DomainCoord c = dcoord(k, g.nd);
        int kc[3] = {c.kx, c.ky, c.kz};
        kc[a] = (dir & 1) ? wrapp(kc[a], g.nd) : wrapm(kc[a], g.nd);
        uint32_t owner = dindex(kc[0], kc[1], kc[2], g.nd) / D;
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

    DevState *st = g.st;
    // launch-start totals (read before any workgroup can publish its first slot,
    // hence before any workgroup can fold its own totals in at the end)
    const uint64_t fired0 = st->fired, nulls0 = st->nulls;
    const int64_t M0 = st->M, B0 = st->B;
    double t = st->t;  // every workgroup advances the same clock
    long long myF = 0, mydM = 0, mydB = 0;  // this thread's share since launch start
    uint32_t rec_index = 0;                  // records produced in this launch
    bool rec_pending = false;
    int prev_colour = -1;

    for (uint64_t n = n0; n < n0 + ncycles; ++n) {
        CycleDraw cd = cycle_draw(g.seed, n);
        const int s = cd.colour;

        // --- step 6 of the previous cycle: wait for the neighbour flips the halo of colour s can see
        if (n > n0) {
            int diff = s ^ prev_colour;
            if (diff && !(diff & (diff - 1))) {
                int a = diff == 1 ? 0 : diff == 2 ? 1 : 2;
                int dir = 2 * a + ((s >> a) & 1);  // below (-) if bit a of s is 0, else above (+)
                const bool all = sh.nbr_cnt[dir] > kMaxNbr;
                const uint32_t cnt = all ? G : sh.nbr_cnt[dir];
                for (uint32_t i = tid; i < cnt; i += nthr) {
                    uint32_t w = all ? i : sh.nbr[dir][i];
                    uint64_t start = now_ticks();
                    while (ld64(&xs.flag[w]) < n) {
                        __builtin_amdgcn_s_sleep(1);
                        if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                            atomicOr(&st->error, kErrFlagTimeout);
                            sh.abort = 1;
                            break;
                        }
                    }
                }
                __syncthreads();
                if (sh.abort) break;
            }
        }
        prev_colour = s;

        // --- steps 1 and 4a: class planes and histograms of the active octants
        Planes<H> pl[P];
#pragma unroll
        for (int pp = 0; pp < P; ++pp) {
            uint32_t ld = (uint32_t)(pp * rows + row);
            uint32_t k = kbase + ld;
            bool valid = ld < nvalid;
            uint32_t m[13];
#pragma unroll
            for (int i = 0; i < 13; ++i) m[i] = 0;
            bin_octant<H>(g, k, s, valid, l, pl[pp], m);
#pragma unroll
            for (int i = 0; i < 13; ++i) m[i] = row_scan(m[i]);
            if (l == 15) {
#pragma unroll
                for (int i = 0; i < 13; ++i) sh.mom[ld][i] = m[i];
            }
            // keep the passes apart: interleaving them only adds live registers
            __builtin_amdgcn_sched_barrier(0);
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

        // --- step 2: R_max over all active octants
        if (tid < 64) {
            double v = 0.0;
            for (uint32_t i = tid; i < D; i += 64) v = fmax(v, sh.rk[i]);
            for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
            // bank n & 1 holds cycles n - 2 and n; the generation bit tells them apart
            uint64_t *bank = xs.slot + (n & 1) * (uint64_t)G;
            const uint64_t parity = ((n >> 1) & 1) << 63;
            if (tid == 0) st64(&bank[gid], double_to_bits(v) | parity);
            // poll every slot until all carry this cycle's parity
            uint64_t start = now_ticks();
            double best = 0.0;
            for (uint32_t base = 0; base < G; base += 64) {
                uint32_t w = base + tid;
                uint64_t sv = parity;
                if (w < G) {
                    sv = ld64(&bank[w]);
                    while ((sv & (1ull << 63)) != parity) {
                        __builtin_amdgcn_s_sleep(1);
                        if (now_ticks() - start > kTimeoutTicks || ld32(&st->error)) {
                            atomicOr(&st->error, kErrBarrierTimeout);
                            sh.abort = 1;
                            break;
                        }
                        sv = ld64(&bank[w]);
                    }
                }
                best = fmax(best, bits_to_double(sv & ~(1ull << 63)));
            }
            for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o));
            if (tid == 0) sh.rmax = best;
        }
        __syncthreads();
        if (sh.abort) break;
        const double Rmax = sh.rmax;

        // pending record of the previous cycle: every workgroup has finished it
        if (rec_pending && gid == 0 && tid == 0 && g.rec_cap) {
            long long F = 0, dM = 0, dB = 0;
            const int64_t *rp = xs.recp + (uint64_t)((rec_index - 1) & 1) * G * 3;
            for (uint32_t w = 0; w < G; ++w) {
                F += (long long)ld64((const uint64_t *)&rp[3 * w]);
                dM += (long long)ld64((const uint64_t *)&rp[3 * w + 1]);
                dB += (long long)ld64((const uint64_t *)&rp[3 * w + 2]);
            }
            spkmc_record r;
            r.cycle = n;  // the state after cycle n - 1
            r.fired = fired0 + (uint64_t)F;
            r.nulls = nulls0 + (uint64_t)g.K * (n - n0) - (uint64_t)F;
            r.t = t;
            r.M = M0 + dM;
            r.B = B0 + dB;
            g.rec[st->rec_count % g.rec_cap] = r;
            st->rec_count += 1;
        }
        rec_pending = false;

        // --- steps 3, 4 and 4b: event or null in every domain, then the flip
#pragma unroll
        for (int pp = 0; pp < P; ++pp) {
            uint32_t ld = (uint32_t)(pp * rows + row);
            uint32_t k = kbase + ld;
            bool valid = ld < nvalid;
            int cs = -1;
            uint32_t j = 0;
            if (valid) {
                U4 dw = philox10((uint32_t)n, (uint32_t)(n >> 32), k, (uint32_t)s, g.seed);
                double target = unit53(dw.x, dw.y) * Rmax;
                // first class whose running sum exceeds the target; none: the null event
                for (int c = 0; c < 14; ++c)
                    if (target < sh.acc[ld][c]) { cs = c; break; }
                if (cs >= 0) j = mul_index(dw.z, sh.hist[ld][cs]);
            }
            // class cs as (spin, n_up pattern): up spin: n_up = a; down spin: n_up = 6 - a
            uint32_t es = 0, e0 = 0, e1 = 0, e2 = 0;
            int a = 0;
            if (cs >= 0) {
                int up = cs >= 7;
                a = cs % 7;
                int v = up ? a : 6 - a;
                es = up ? 0xFFFFFFFFu : 0u;
                e0 = (v & 1) ? 0xFFFFFFFFu : 0u;
                e1 = (v & 2) ? 0xFFFFFFFFu : 0u;
                e2 = (v & 4) ? 0xFFFFFFFFu : 0u;
            }
            constexpr int WPL = Planes<H>::W;
            uint32_t mk[WPL];
            uint32_t cnt = 0;
#pragma unroll
            for (int p = 0; p < WPL; ++p) {
                uint32_t miss = (pl[pp].S[p] ^ es) | (pl[pp].b0[p] ^ e0) | (pl[pp].b1[p] ^ e1) | (pl[pp].b2[p] ^ e2);
                mk[p] = cs >= 0 ? ~miss : 0u;
                cnt += __builtin_popcount(mk[p]);
            }
            // inclusive prefix over the 16 lanes of the row (canonical order = lane order)
            uint32_t incl = row_scan(cnt);
            uint32_t excl = incl - cnt;
            if (cs >= 0 && j >= excl && j < incl) {
                uint32_t r = j - excl;
                int wsel = 0;
#pragma unroll
                for (int p = 0; p < WPL; ++p) {
                    uint32_t c = __builtin_popcount(mk[p]);
                    if (wsel == p && r >= c) { r -= c; wsel = p + 1; }
                }
                uint32_t msk = 0;
#pragma unroll
                for (int p = 0; p < WPL; ++p)
                    if (p == wsel) msk = mk[p];
                for (uint32_t i = 0; i < r; ++i) msk &= msk - 1;
                if (msk == 0) {  // the counts disagree with the masks: report, flip nothing
                    atomicOr(&st->error, kErrSelect);
                    continue;
                }
                int bit = __builtin_ctz(msk);
                uint32_t wq = (uint32_t)(l * WPL + wsel);  // word index inside the octant
                uint32_t q = wq * 32 + (uint32_t)bit;
                uint32_t *A = g.A + ((uint64_t)k * 8 + s) * g.wpo;
                uint32_t old = flip_word(A + wq, 1u << bit);
                int sold = ((old >> bit) & 1u) ? 1 : -1;
                uint32_t lx = q % H, ly = (q / H) % H, lz = q / (H * H);
                uint32_t *F = g.F + ((uint64_t)k * 8 + s) * g.fwpo;
                const uint32_t e = H - 1, h2 = H * H;
                if (lx == 0) { uint32_t b = ly + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
                if (lx == e) { uint32_t b = h2 + ly + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
                if (ly == 0) { uint32_t b = 2 * h2 + lx + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
                if (ly == e) { uint32_t b = 3 * h2 + lx + H * lz; flip_word(F + (b >> 5), 1u << (b & 31)); }
                if (lz == 0) { uint32_t b = 4 * h2 + lx + H * ly; flip_word(F + (b >> 5), 1u << (b & 31)); }
                if (lz == e) { uint32_t b = 5 * h2 + lx + H * ly; flip_word(F + (b >> 5), 1u << (b & 31)); }
                myF += 1;
                mydM += -2 * sold;
                mydB += 12 - 4 * a;
            }
        }

        // --- step 5: the clock, identical in every workgroup
        {
            double dt = -log(cd.ut) / (8.0 * Rmax);
            t = t + dt;
        }

        // flips complete, then publish them (step 6)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();

        const bool record = obs_every && ((n + 1) % obs_every) == 0;
        if (record || n + 1 == n0 + ncycles) {
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
                if (n + 1 == n0 + ncycles) {
                    // end of the launch: fold this workgroup's share into the totals
                    atomicAdd((unsigned long long *)&st->fired, (unsigned long long)F);
                    atomicAdd((unsigned long long *)&st->nulls, (unsigned long long)((long long)nvalid * (long long)ncycles - F));
                    atomicAdd((unsigned long long *)&st->M, (unsigned long long)dM);
                    atomicAdd((unsigned long long *)&st->B, (unsigned long long)dB);
                } else {
                    int64_t *rp = xs.recp + (uint64_t)(rec_index & 1) * G * 3;
                    st64((uint64_t *)&rp[3 * gid], (uint64_t)F);
                    st64((uint64_t *)&rp[3 * gid + 1], (uint64_t)dM);
                    st64((uint64_t *)&rp[3 * gid + 2], (uint64_t)dB);
                }
            }
            if (record && n + 1 != n0 + ncycles) {
                rec_pending = true;
                rec_index += 1;
            }
        }
        if (tid == 0) {
            __builtin_amdgcn_s_waitcnt(0);
            st64(&xs.flag[gid], n + 1);
        }
    }
    if (gid == 0 && tid == 0) {
        st->t = t;
        st->cycle = n0 + ncycles;
    }
}

// Before a launch: slots carry the parity of the previous cycle, flags the start cycle.
__global__ void k_persistent_prep(PersistScratch xs, uint32_t G, uint64_t n0) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G) {
        // bank b first serves cycle nb (n0 or n0 + 1, nb & 1 == b): mark it "not yet"
        for (uint64_t nb = n0; nb < n0 + 2; ++nb) xs.slot[(nb & 1) * G + i] = (((nb >> 1) + 1) & 1) << 63;
        xs.flag[i] = n0;
    }
}

// After a launch: the record of the last cycle, from the final totals.
__global__ void k_persistent_finish(Geom g, uint64_t n_end, uint32_t obs_every) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState *st = g.st;
    if (obs_every && (n_end % obs_every) == 0 && g.rec_cap) {
        spkmc_record r;
        r.cycle = n_end;
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
// host side
// ---------------------------------------------------------------------------
// Launch shapes: h = 16 keeps 4 passes of 32 domains in registers with 512
// threads (two waves per SIMD, 256 registers each); h = 8 needs 4 registers per
// pass and runs 1024 threads.
template <int H, int P, int BLOCK>
static void *kernel_ptr() {
    return reinterpret_cast<void *>(&k_persistent<H, P, BLOCK>);
}
static void *select_kernel(int h, int P, int block) {
    if (h == 16) {
        if (block == 512) return P == 1 ? kernel_ptr<16, 1, 512>() : P == 2 ? kernel_ptr<16, 2, 512>() : kernel_ptr<16, 4, 512>();
        return nullptr;
    }
    if (block == 1024) return P == 1 ? kernel_ptr<8, 1, 1024>() : P == 2 ? kernel_ptr<8, 2, 1024>() : kernel_ptr<8, 4, 1024>();
    if (block == 256) return P == 1 ? kernel_ptr<8, 1, 256>() : nullptr;
    return nullptr;
}

bool persistent_supported(const Geom &g, const spkmc_params &p, std::string &why) {
    if (g.layout != SPKMC_LAYOUT_PACKED) { why = "needs the PACKED layout"; return false; }
    if (g.h != 8 && g.h != 16) { why = "needs an octant edge of 8 or 16 (domain 16 or 32)"; return false; }
    if (p.wg_domains && p.wg_domains != (g.h == 16 ? 32 : 64) * (p.wg_domains / (g.h == 16 ? 32 : 64))) {
        why = "wg_domains must be 32, 64 or 128 (h = 16) or 64, 128 or 256 (h = 8)";
        return false;
    }
    return true;
}

hipError_t persistent_configure(const Geom &g, const spkmc_params &p, int &grid, int &block, int &wg_domains) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int rows = g.h == 16 ? 32 : 64;  // domains per pass
    int P = 0;
    block = rows * 16;
    if (p.wg_domains) {
        for (int Pc : {1, 2, 4})
            if (rows * Pc == p.wg_domains) P = Pc;
        if (!P) return hipErrorInvalidValue;
    } else {
        // the fewest passes that keep every workgroup resident (one per CU at most)
        P = 1;
        while (P < 4 && (g.K + (uint64_t)rows * P - 1) / ((uint64_t)rows * P) > (uint64_t)cus) P <<= 1;
    }
    void *kern = select_kernel(g.h, P, block);
    if (!kern) return hipErrorInvalidValue;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, 0);
    if (e != hipSuccess) return e;
    uint64_t D = (uint64_t)rows * P;
    uint64_t G = (g.K + D - 1) / D;
    if (occ <= 0 || G > (uint64_t)occ * cus || G > (uint64_t)kMaxGrid) return hipErrorCooperativeLaunchTooLarge;
    grid = (int)G;
    wg_domains = (int)D;
    return hipSuccess;
}

static PersistScratch scratch_of(const Geom &g, int G) {
    PersistScratch xs;
    xs.slot = g.sync;
    xs.flag = g.sync + 2 * (uint64_t)G;
    xs.recp = reinterpret_cast<int64_t *>(g.sync + 3 * (uint64_t)G);
    return xs;
}

hipError_t launch_persistent(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid, int block,
                             int wg_domains, hipStream_t stream) {
    PersistScratch xs = scratch_of(g, grid);
    int P = wg_domains / (block / 16);
    void *kern = select_kernel(g.h, P, block);
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persistent_prep, dim3((grid + 255) / 256), dim3(256), 0, stream, xs, (uint32_t)grid, n0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    Geom gg = g;
    void *args[] = {&gg, &xs, &n0, &ncycles, &obs_every};
    e = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(block), args, 0, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_persistent_finish, dim3(1), dim3(64), 0, stream, gg, n0 + ncycles, obs_every);
    return hipGetLastError();
}

}  // namespace spkmc
