// kernels_rows.hip -- the per-cycle engine's row kernels of the gfx950 spkMC
// library (PACKED, octant edge 8 or 16): one cycle in two launches with the
// persistent kernel's rows and passes, for lattices whose lines do not fit the
// device at once (persistent_common.hpp holds the shared binning, selection and
// flip code).
#include <string>

#include "api_internal.hpp"
#include "persistent_common.hpp"

namespace spkmc {

// ---------------------------------------------------------------------------
// The per-cycle engine's row kernels (PACKED, octant edge 8 or 16): one cycle in
// two launches, for lattices of any size.  k_rows_bin bins every line with the
// persistent kernel's rows and passes (step 1) and takes the maximum (step 2)
// into st->rmax[0]; k_rows_select derives the class planes again, draws,
// selects and flips (steps 3, 4, 4b; step 6 is the launch boundary); the
// per-cycle k_finalize keeps the clock, the counters and the records (step 5).
constexpr int kRowsPasses = 4;  // passes of the row kernels (128 or 256 lines per workgroup)

struct RowsShared {
    alignas(16) uint32_t zbuf[64][kRowHalo];  // per row: the six halo faces (8 words each), zeros (8)
    uint32_t nbdom[kMaxWgDomains][6];  // per line: its domain's six neighbour domains
    double acc[kMaxWgDomains][14];     // per line: running FP64 sums of the frequency line
    uint32_t hist[kMaxWgDomains][14];  // per line: class counts
    uint32_t selq[kMaxWgDomains];      // per line: (class << 12) | site q, or kNoEvent
    unsigned long long wmax;           // the workgroup's largest line (FP64 bits)
    long long red[3][16];
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
    if (l < 8) sh.zbuf[row][48 + l] = 0;
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
    if (l < 8) sh.zbuf[row][48 + l] = 0;
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
        flip_site<H>(g, rg.dom(rg.kbase + t), rg.oct(rg.kbase + t, s), q, sh.nbdom[t]);
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

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
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

hipError_t launch_cycle_rows(const Geom &g, uint64_t n, hipStream_t stream) {
    if (!rows_supported(g)) return hipErrorInvalidValue;
    return g.h == 16 ? launch_rows<16, 512, kRowsPasses>(g, n, stream) : launch_rows<8, 1024, kRowsPasses>(g, n, stream);
}

}  // namespace spkmc
