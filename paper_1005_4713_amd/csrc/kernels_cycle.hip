// kernels_cycle.hip -- state set-up kernels and the per-cycle ("CYCLE" engine)
// kernels of the gfx950 spkMC library.
//
// One cycle (Sec. 3.1 steps 1-6, Sec. 3.2 steps 4a/4b) is three launches:
//   k_bin      one workgroup per frequency line (an active octant): class
//              histogram (step 1), its FP64 frequency line R_k, device-wide
//              max (step 2);
//   k_select   one wavefront per frequency line: draw, frequency-line walk with the
//              null event last (steps 3, 4, 4b), canonical-order prefix select
//              of the site with wavefront ballots, flip (step 6 is the kernel
//              boundary);
//   k_finalize one thread: clock (step 5), counters, observation record.
// These kernels are generic over the spin layout and serve as the reference
// launch shape for the persistent engine.
#include "api_internal.hpp"
#include "spkmc_device.hpp"

namespace spkmc {

// --------------------------------------------------------------------------- set-up
__global__ void k_init_int8(Geom g, int init) {
    uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 128-site block
    uint64_t first = b << 7;
    if (first >= g.N) return;
    U4 w = philox10((uint32_t)b, (uint32_t)(b >> 32), 0xFFFFFFFEu, 0xFFFFFFFEu, g.seed);
    uint32_t words[4] = {w.x, w.y, w.z, w.w};
    for (int i = 0; i < 128 && first + i < g.N; ++i) {
        int v = init == SPKMC_INIT_UP ? 1 : init == SPKMC_INIT_DOWN ? -1 : ((words[i >> 5] >> (i & 31)) & 1u) ? 1 : -1;
        g.spin8[first + i] = (int8_t)v;
    }
}

// One thread per packed word: 32 consecutive canonical sites of one octant.
__global__ void k_init_packed(Geom g, int init) {
    uint64_t wi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t total = (uint64_t)g.K * 8 * g.wpo;
    if (wi >= total) return;
    uint64_t oct = wi / g.wpo;
    uint32_t k = (uint32_t)(oct >> 3);
    int s = (int)(oct & 7);
    uint32_t q0 = (uint32_t)(wi % g.wpo) * 32;
    int ox, oy, oz;
    octant_origin(g, k, s, ox, oy, oz);
    uint32_t word = 0;
    if (init == SPKMC_INIT_UP) {
        word = 0xFFFFFFFFu;
    } else if (init == SPKMC_INIT_RANDOM) {
        uint64_t cached = ~0ull;
        U4 w{0, 0, 0, 0};
        for (int b = 0; b < 32; ++b) {
            uint32_t q = q0 + b;
            int lx = (int)(q % g.h), ly = (int)((q / g.h) % g.h), lz = (int)(q / g.h2);
            uint64_t i = (uint64_t)(ox + lx) + (uint64_t)g.L * ((uint64_t)(oy + ly) + (uint64_t)g.L * (uint64_t)(oz + lz));
            uint64_t blk = i >> 7;
            if (blk != cached) {
                w = philox10((uint32_t)blk, (uint32_t)(blk >> 32), 0xFFFFFFFEu, 0xFFFFFFFEu, g.seed);
                cached = blk;
            }
            uint32_t src = ((i >> 5) & 3) == 0 ? w.x : ((i >> 5) & 3) == 1 ? w.y : ((i >> 5) & 3) == 2 ? w.z : w.w;
            word |= ((src >> (i & 31)) & 1u) << b;
        }
    }
    g.A[wi] = word;
}

// The octant across face `a` (axis) of octant (k, s): below (side 0) or above
// (side 1), in this domain or the neighbour domain (periodic).
__device__ inline uint64_t octant_across(const Geom &g, uint32_t k, int s, int a, int side) {
    const uint32_t nd = (uint32_t)g.nd;
    uint32_t kc[3] = {k % nd, (k / nd) % nd, k / (nd * nd)};
    const int sa = (s >> a) & 1;
    if (sa == side) kc[a] = side ? (kc[a] + 1 == nd ? 0 : kc[a] + 1) : (kc[a] == 0 ? nd - 1 : kc[a] - 1);
    return ((uint64_t)(kc[0] + nd * (kc[1] + nd * kc[2]))) * 8 + (uint64_t)(s ^ (1 << a));
}

// Halo copies of every octant, rebuilt from the packed spins.  Halo slot f of
// an octant: x below, x above, y below, y above, z below, z above: the layer at
// local coordinate h - 1 of the octant below along the axis (slots 0, 2, 4) or
// layer 0 of the octant above (1, 3, 5).  Inside a slot the bit index is
// (ly + h lz) for x, (lx + h lz) for y, (lx + h ly) for z.
__global__ void k_build_faces(Geom g) {
    uint64_t fw = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t total = (uint64_t)g.K * 8 * g.fwpo;
    if (fw >= total) return;
    uint64_t oct = fw / g.fwpo;
    const uint32_t k = (uint32_t)(oct >> 3);
    const int s = (int)(oct & 7u);
    uint32_t base_bit = (uint32_t)(fw % g.fwpo) * 32;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
        uint32_t fb = base_bit + b;
        uint32_t f = fb / g.h2, idx = fb % g.h2;
        const int a = (int)(f >> 1), side = (int)(f & 1);
        const uint32_t *srcA = g.A + octant_across(g, k, s, a, side) * g.wpo;
        uint32_t u = idx % g.h, v = idx / g.h, e = side ? 0 : g.h - 1;
        uint32_t lx, ly, lz;
        if (a == 0) { lx = e; ly = u; lz = v; }
        else if (a == 1) { lx = u; ly = e; lz = v; }
        else { lx = u; ly = v; lz = e; }
        uint32_t q = lx + g.h * (ly + g.h * lz);
        word |= ((srcA[q >> 5] >> (q & 31)) & 1u) << b;
    }
    g.F[fw] = word;
}

// M and B of the whole lattice (each bond once: +x, +y, +z of every site).
template <class S>
__global__ void k_observables(Geom g) {
    __shared__ long long shM[256], shB[256];
    long long m = 0, b = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += (uint64_t)gridDim.x * blockDim.x) {
        int x = (int)(i % g.L), y = (int)((i / g.L) % g.L), z = (int)(i / ((uint64_t)g.L * g.L));
        int s = S::get(g, x, y, z);
        m += s;
        b += s * (S::get(g, x + 1 == g.L ? 0 : x + 1, y, z) + S::get(g, x, y + 1 == g.L ? 0 : y + 1, z) +
                  S::get(g, x, y, z + 1 == g.L ? 0 : z + 1));
    }
    shM[threadIdx.x] = m;
    shB[threadIdx.x] = b;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            shM[threadIdx.x] += shM[threadIdx.x + o];
            shB[threadIdx.x] += shB[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&g.st->M, (unsigned long long)shM[0]);
        atomicAdd((unsigned long long *)&g.st->B, (unsigned long long)shB[0]);
    }
}

// --------------------------------------------------------------------------- cycle
constexpr unsigned kCycleMaxGrid = 1u << 20;  // workgroups of one generic per-cycle launch
// Frequency line f of a cycle: domain f / lpd, octant = the colour (eight
// colours) or the (f mod 4)-th octant of the colour's parity (two colours).
__device__ __forceinline__ void line_of(const Geom &g, uint32_t f, int colour, uint32_t &k, int &s) {
    if (g.lpd == 1) {
        k = f;
        s = colour;
    } else {
        k = f >> 2;
        s = two_colour_octant(colour, f & 3u);
    }
}

template <class S>
__device__ __forceinline__ void bin_octant(const Geom &g, uint32_t k, int s, uint32_t *cnt) {
    int ox, oy, oz;
    octant_origin(g, k, s, ox, oy, oz);
    for (uint32_t q = threadIdx.x; q < g.h3; q += blockDim.x) {
        int x = ox + (int)(q % g.h), y = oy + (int)((q / g.h) % g.h), z = oz + (int)(q / g.h2);
        int sp = S::get(g, x, y, z);
        int c = (sp > 0 ? 7 : 0) + aligned_count<S>(g, x, y, z, sp);
        atomicAdd(&cnt[c], 1u);
    }
}

// Step 1 and the device-wide max of step 2.  One workgroup per frequency line
// (lines f = blockIdx.x, blockIdx.x + gridDim.x, ... when the lines outnumber the
// grid).  RMAX_ALL: the workgroup also bins the inactive octants each line
// stands for (the other seven with eight colours, octant s ^ 1 with two) into
// the maximum; RMAX_BOUND: no maximum is taken.
template <class S>
__global__ void k_bin(Geom g, uint64_t n) {
    __shared__ uint32_t cnt[16];
    const uint32_t lines = g.K * g.lpd;  // < 2^31 (checked at set-up)
    const bool two = g.lpd == 4;
    const CycleDraw cd = cycle_draw(g.seed, n, two);
    double wmax = 0.0;  // thread 0: the largest line of this workgroup
    for (uint32_t f = blockIdx.x; f < lines; f += gridDim.x) {
        uint32_t k;
        int s;
        line_of(g, f, cd.colour, k, s);
        __syncthreads();  // the previous line's counts are read
        if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
        __syncthreads();
        bin_octant<S>(g, k, s, cnt);
        __syncthreads();
        double Rk = 0.0;
        if (threadIdx.x == 0) {
            Rk = line_total(cnt, g.r);
            g.Rk[f] = Rk;
            for (int c = 0; c < 16; ++c) g.hist[(uint64_t)f * 16 + c] = c < 14 ? cnt[c] : 0;
        }
        if (g.variant & SPKMC_VARIANT_RMAX_ALL) {
            for (int o = 0; o < 8; ++o) {
                if (o == s || (two && o != (s ^ 1))) continue;
                __syncthreads();
                if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
                __syncthreads();
                bin_octant<S>(g, k, o, cnt);
                __syncthreads();
                if (threadIdx.x == 0) {
                    double Ro = line_total(cnt, g.r);
                    if (Ro > Rk) Rk = Ro;
                }
            }
        }
        if (Rk > wmax) wmax = Rk;
    }
    if (threadIdx.x == 0 && !(g.variant & SPKMC_VARIANT_RMAX_BOUND) && blockIdx.x < lines)
        atomicMax((unsigned long long *)&g.st->rmax[0], (unsigned long long)double_to_bits(wmax));
}

// Steps 3, 4, 4b and the flip.  One 64-lane wavefront per frequency line, four
// per workgroup (lines f, f + 4 gridDim.x, ... when the lines outnumber the grid).
template <class S>
__global__ void __launch_bounds__(256) k_select(Geom g, uint64_t n) {
    __shared__ long long part[4][3];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t lines = g.K * g.lpd;  // < 2^31 (checked at set-up)
    const CycleDraw cd = cycle_draw(g.seed, n, g.lpd == 4);
    const double Rmax = (g.variant & SPKMC_VARIANT_RMAX_BOUND) ? g.rbound : bits_to_double(g.st->rmax[0]);
    long long fired = 0, dM = 0, dB = 0;
    for (uint32_t f = blockIdx.x * 4 + wave; f < lines; f += gridDim.x * 4) {
        uint32_t k;
        int so;
        line_of(g, f, cd.colour, k, so);
        U4 dw = philox10((uint32_t)n, (uint32_t)(n >> 32), k, (uint32_t)so, g.seed);
        double target = unit53(dw.x, dw.y) * Rmax;
        uint32_t cnt[14];
        for (int c = 0; c < 14; ++c) cnt[c] = g.hist[(uint64_t)f * 16 + c];
        int cs = line_select(cnt, g.r, target);
        if (cs >= 0) {
            uint32_t j = mul_index(dw.z, cnt[cs]);
            int ox, oy, oz;
            octant_origin(g, k, so, ox, oy, oz);
            for (uint32_t q0 = 0; q0 < g.h3; q0 += 64) {
                uint32_t q = q0 + lane;
                int x = 0, y = 0, z = 0, s = 0, a = 0;
                bool hit = false;
                if (q < g.h3) {
                    x = ox + (int)(q % g.h);
                    y = oy + (int)((q / g.h) % g.h);
                    z = oz + (int)(q / g.h2);
                    s = S::get(g, x, y, z);
                    a = aligned_count<S>(g, x, y, z, s);
                    hit = ((s > 0 ? 7 : 0) + a) == cs;
                }
                uint64_t m = __ballot(hit);
                uint32_t c = (uint32_t)__popcll(m);
                if (j < c) {
                    // lane whose rank among the hits is j
                    uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                    if (hit && below == j) {
                        if (g.layout == SPKMC_LAYOUT_INT8) {
                            g.spin8[(int64_t)x + (int64_t)g.L * ((int64_t)y + (int64_t)g.L * z)] = (int8_t)(-s);
                        } else {
                            uint64_t bit = ((uint64_t)k * 8 + (uint64_t)so) * g.h3 + q;
                            atomicXor(&g.A[bit >> 5], 1u << (bit & 31));
                            // the halo copies of the octants across the boundary layers it lies on
                            const uint32_t c3[3] = {q % g.h, (q / g.h) % g.h, q / g.h2};
                            for (int a = 0; a < 3; ++a) {
                                if (c3[a] != 0 && c3[a] != g.h - 1) continue;
                                for (int side = 0; side < 2; ++side) {
                                    // layer 0 is in the halo above of the octant below (side 0)
                                    if (c3[a] != (side ? g.h - 1 : 0)) continue;
                                    const uint32_t u = a == 0 ? c3[1] : c3[0], v = a == 2 ? c3[1] : c3[2];
                                    const uint32_t b = (uint32_t)(2 * a + (side ? 0 : 1)) * g.h2 + u + g.h * v;
                                    uint32_t *Ft = g.F + octant_across(g, k, so, a, side) * g.fwpo;
                                    atomicXor(&Ft[b >> 5], 1u << (b & 31));
                                }
                            }
                        }
                        fired += 1;
                        dM += -2 * s;
                        dB += 12 - 4 * a;
                    }
                    break;
                }
                j -= c;
            }
        }
    }
    // wavefront sums of the lanes that flipped
    for (int o = 32; o > 0; o >>= 1) {
        fired += __shfl_xor(fired, o);
        dM += __shfl_xor(dM, o);
        dB += __shfl_xor(dB, o);
    }
    if (lane == 0) {
        part[wave][0] = fired;
        part[wave][1] = dM;
        part[wave][2] = dB;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long f = 0, m = 0, b = 0;
        for (int w = 0; w < 4; ++w) {
            f += part[w][0];
            m += part[w][1];
            b += part[w][2];
        }
        if (f) atomicAdd((unsigned long long *)&g.st->acc_fired[0], (unsigned long long)f);
        if (m) atomicAdd((unsigned long long *)&g.st->acc_dM[0], (unsigned long long)m);
        if (b) atomicAdd((unsigned long long *)&g.st->acc_dB[0], (unsigned long long)b);
    }
}

// Step 5 and the bookkeeping of cycle n.
__global__ void k_finalize(Geom g, uint64_t n, uint32_t obs_every) {
    if (threadIdx.x == 0) finalize_cycle(g, n, obs_every);
}

// --------------------------------------------------------------------------- host launchers
hipError_t launch_init(const Geom &g, int init, hipStream_t stream) {
    if (g.layout == SPKMC_LAYOUT_INT8) {
        uint64_t blocks128 = (g.N + 127) / 128;
        hipLaunchKernelGGL(k_init_int8, dim3((unsigned)((blocks128 + 255) / 256)), dim3(256), 0, stream, g, init);
    } else {
        uint64_t words = (uint64_t)g.K * 8 * g.wpo;
        hipLaunchKernelGGL(k_init_packed, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream, g, init);
    }
    return hipGetLastError();
}

hipError_t launch_faces(const Geom &g, hipStream_t stream) {
    if (g.layout != SPKMC_LAYOUT_PACKED) return hipSuccess;
    uint64_t fwords = (uint64_t)g.K * 8 * g.fwpo;
    hipLaunchKernelGGL(k_build_faces, dim3((unsigned)((fwords + 255) / 256)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_observables(const Geom &g, hipStream_t stream) {
    uint64_t blocks = (g.N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (g.layout == SPKMC_LAYOUT_INT8)
        hipLaunchKernelGGL(k_observables<Int8Spins>, dim3((unsigned)blocks), dim3(256), 0, stream, g);
    else
        hipLaunchKernelGGL(k_observables<PackedSpins>, dim3((unsigned)blocks), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_cycle(const Geom &g, uint64_t n, uint32_t obs_every, hipStream_t stream, bool slab) {
    if (slab) {
        // PACKED lattices with octant edge 16: the per-cycle slab kernels (their
        // counts binned at the start of the run), then step 5 here
        hipError_t e = launch_cycle_slab(g, n, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, stream, g, n, obs_every);
        return hipGetLastError();
    }
    if (rows_supported(g)) {
        // PACKED lattices with octant edge 8 or 16: the row kernels, then step 5 here
        hipError_t e = launch_cycle_rows(g, n, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, stream, g, n, obs_every);
        return hipGetLastError();
    }
    // grids capped well below the 2^32 work-items of one dispatch; the kernels
    // stride over the remaining lines
    const unsigned bin_block = g.h3 >= 256 ? 256 : 64;
    const unsigned lines = g.K * g.lpd;
    const unsigned bin_blocks = lines < kCycleMaxGrid ? lines : kCycleMaxGrid;
    const unsigned sel_blocks = (lines + 3) / 4 < kCycleMaxGrid ? (lines + 3) / 4 : kCycleMaxGrid;
    if (g.layout == SPKMC_LAYOUT_INT8) {
        hipLaunchKernelGGL(k_bin<Int8Spins>, dim3(bin_blocks), dim3(bin_block), 0, stream, g, n);
        hipLaunchKernelGGL(k_select<Int8Spins>, dim3(sel_blocks), dim3(256), 0, stream, g, n);
    } else {
        hipLaunchKernelGGL(k_bin<PackedSpins>, dim3(bin_blocks), dim3(bin_block), 0, stream, g, n);
        hipLaunchKernelGGL(k_select<PackedSpins>, dim3(sel_blocks), dim3(256), 0, stream, g, n);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, stream, g, n, obs_every);
    return hipGetLastError();
}

}  // namespace spkmc
