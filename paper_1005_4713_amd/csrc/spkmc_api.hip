// spkmc_api.hip -- the C ABI declared in include/spkmc.h (host side).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "api_internal.hpp"

using namespace spkmc;

static thread_local std::string g_last_error = "no error";

static spkmc_status fail(spkmc_ctx *c, spkmc_status st, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (st == SPKMC_E_DEVICE) c->failed = true;
    } else {
        g_last_error = msg;
    }
    return st;
}

static spkmc_status hip_fail(spkmc_ctx *c, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, SPKMC_E_DEVICE, m);
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Host FP64 rate table: class c -> spin sign, aligned count a; flip energy
// change dE = 2 J (2a - 6) + 2 H s from eq. 1; Glauber 1 / (1 + exp(beta dE))
// or Metropolis min(1, exp(-beta dE)).  Evaluated without FMA contraction so the
// values are reproducible bit for bit.
static int make_rates(const spkmc_params *p, double out[14]) {
    if (!(p->T > 0.0) || !isfinite(p->T) || !isfinite(p->J) || !isfinite(p->H)) return -1;
    double beta = 1.0 / p->T;
    for (int c = 0; c < 14; ++c) {
        int sgn = c >= 7 ? 1 : -1;
        int a = c % 7;
        double dE = 2.0 * p->J * (double)(2 * a - 6) + 2.0 * p->H * (double)sgn;
        double x = beta * dE;
        double r = p->rates == SPKMC_RATES_GLAUBER ? 1.0 / (1.0 + exp(x)) : (dE <= 0.0 ? 1.0 : exp(-x));
        if (!(r > 0.0) || !isfinite(r)) return -2;
        out[c] = r;
    }
    return 0;
}

struct LayoutPlan {
    size_t off_rates, off_rec, off_Rk, off_hist, off_flip, off_sync, off_dh, off_sc, off_spin, off_F, total, spin_bytes;
};

static bool validate(const spkmc_params *p, std::string &why) {
    if (!p) { why = "params is NULL"; return false; }
    if (p->struct_size != sizeof(spkmc_params)) { why = "struct_size does not match sizeof(spkmc_params)"; return false; }
    if (p->variant & ~(uint32_t)(SPKMC_VARIANT_RMAX_ALL | SPKMC_VARIANT_TWO_COLOURS | SPKMC_VARIANT_RMAX_BOUND)) {
        why = "unknown variant bits";
        return false;
    }
    if ((p->variant & SPKMC_VARIANT_RMAX_ALL) && (p->variant & SPKMC_VARIANT_RMAX_BOUND)) {
        why = "RMAX_ALL and RMAX_BOUND exclude each other";
        return false;
    }
    if (p->L < 2) { why = "L must be >= 2"; return false; }
    if (p->domain < 2 || (p->domain & 1)) { why = "domain edge must be even and >= 2"; return false; }
    if (p->L % p->domain) { why = "L must be a multiple of the domain edge"; return false; }
    if (p->L > 4096) { why = "L above 4096 is not supported"; return false; }
    // octant sites and word counts are 32-bit: h^3 < 2^31
    if (p->domain > 2048) { why = "domain edge above 2048 is not supported (octants of 2^31 sites or more)"; return false; }
    {
        const uint64_t nd = (uint64_t)(p->L / p->domain);
        const uint64_t lines = nd * nd * nd * ((p->variant & SPKMC_VARIANT_TWO_COLOURS) ? 4 : 1);
        if (lines >= (1ull << 31)) {
            why = "more than 2^31 - 1 frequency lines (domains times lines per domain): use larger domains";
            return false;
        }
    }
    if (p->rates != SPKMC_RATES_GLAUBER && p->rates != SPKMC_RATES_METROPOLIS) { why = "unknown rates"; return false; }
    if (p->init < 0 || p->init > 2) { why = "unknown init"; return false; }
    if (p->layout != SPKMC_LAYOUT_INT8 && p->layout != SPKMC_LAYOUT_PACKED) { why = "unknown layout"; return false; }
    if (p->engine < 0 || p->engine > 4) { why = "unknown engine"; return false; }
    if (p->wg_domains < 0) { why = "wg_domains must be >= 0"; return false; }
    int h = p->domain / 2;
    if (p->layout == SPKMC_LAYOUT_PACKED && (h % 4)) { why = "PACKED layout needs the octant edge (domain/2) to be a multiple of 4"; return false; }
    double r[14];
    int rc = make_rates(p, r);
    if (rc == -1) { why = "T must be > 0 and J, H, T finite"; return false; }
    if (rc == -2) { why = "a rate is 0 or not finite (temperature too low for FP64)"; return false; }
    return true;
}

static LayoutPlan plan(const spkmc_params *p) {
    LayoutPlan lp;
    uint64_t L = (uint64_t)p->L, N = L * L * L, nd = L / (uint64_t)p->domain, K = nd * nd * nd;
    uint64_t h = (uint64_t)p->domain / 2;
    size_t o = 256;  // DevState
    lp.off_rates = o; o += 256;
    lp.off_rec = o; o = align256(o + (size_t)p->record_cap * sizeof(spkmc_record));
    const uint64_t lines = K * ((p->variant & SPKMC_VARIANT_TWO_COLOURS) ? 4 : 1);
    lp.off_Rk = o; o = align256(o + lines * 8);
    lp.off_hist = o; o = align256(o + lines * 64);
    lp.off_flip = o; o = align256(o + K * 8);
    // persistent engine: slots, flags and record partials of its workgroups, and
    // the class changes its workgroups push to one another (PACKED)
    lp.off_sync = o; o = align256(o + persistent_scratch_words(lines) * 8);
    lp.off_dh = o;
    if (p->layout == SPKMC_LAYOUT_PACKED) o = align256(o + K * 16 * 8);
    // slab engine: 28 words of slab class counts per octant (PACKED, h = 16)
    lp.off_sc = o;
    if (p->layout == SPKMC_LAYOUT_PACKED && h == 16) o = align256(o + K * 8 * 28 * 4);
    lp.off_spin = o;
    if (p->layout == SPKMC_LAYOUT_INT8) {
        o = align256(o + N);
        lp.off_F = 0;
    } else {
        o = align256(o + N / 8);
        lp.off_F = o;
        o = align256(o + K * 8 * 6 * h * h / 8);
    }
    lp.spin_bytes = o - lp.off_spin;
    lp.total = o;
    return lp;
}

void spkmc::obs_from_state(const spkmc_params &p, uint64_t N, const DevState &st, spkmc_obs *out) {
    out->rec.cycle = st.cycle;
    out->rec.fired = st.fired;
    out->rec.nulls = st.nulls;
    out->rec.t = st.t;
    out->rec.M = st.M;
    out->rec.B = st.B;
    out->E = -p.J * (double)st.B - p.H * (double)st.M;  // eq. 1
    out->m = (double)st.M / (double)N;                    // eq. 4
    uint64_t tot = st.fired + st.nulls;
    out->ur = tot ? (double)st.fired / (double)tot : 0.0;
}

#pragma GCC visibility push(default)
extern "C" {

size_t spkmc_state_bytes(const spkmc_params *p) {
    std::string why;
    if (!validate(p, why)) {
        g_last_error = why;
        return 0;
    }
    return plan(p).total;
}

spkmc_status spkmc_rate_table(const spkmc_params *p, double out[14]) {
    std::string why;
    if (!out) return fail(nullptr, SPKMC_E_INVAL, "out is NULL");
    if (!validate(p, why)) return fail(nullptr, SPKMC_E_INVAL, why);
    make_rates(p, out);
    return SPKMC_OK;
}

spkmc_status spkmc_init(const spkmc_params *p, void *dev_buf, size_t dev_bytes, void *hip_stream, spkmc_ctx **out) {
    if (!out) return fail(nullptr, SPKMC_E_INVAL, "out is NULL");
    *out = nullptr;
    spkmc_ctx *c = new (std::nothrow) spkmc_ctx();
    if (!c) return fail(nullptr, SPKMC_E_NOMEM, "cannot allocate context");
    *out = c;
    c->failed = false;
    c->cycle = 0;
    c->primed_grid = 0;
    std::string why;
    if (!validate(p, why)) return fail(c, SPKMC_E_INVAL, why);
    c->p = *p;
    LayoutPlan lp = plan(p);
    if (!dev_buf) return fail(c, SPKMC_E_INVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf) & 255) return fail(c, SPKMC_E_INVAL, "dev_buf must be 256-byte aligned");
    if (dev_bytes < lp.total) {
        char m[160];
        snprintf(m, sizeof m, "dev_bytes %zu < required %zu", dev_bytes, lp.total);
        return fail(c, SPKMC_E_RANGE, m);
    }
    c->stream = (hipStream_t)hip_stream;
    c->dev = (char *)dev_buf;
    c->dev_bytes = dev_bytes;
    Geom &g = c->g;
    memset(&g, 0, sizeof g);
    g.L = p->L;
    g.d = p->domain;
    g.h = p->domain / 2;
    g.nd = p->L / p->domain;
    g.layout = p->layout;
    g.K = (uint32_t)((uint64_t)g.nd * g.nd * g.nd);
    g.N = (uint64_t)p->L * p->L * p->L;
    g.h2 = (uint32_t)(g.h * g.h);
    g.h3 = g.h2 * (uint32_t)g.h;
    g.wpo = g.h3 / 32;
    g.fwpo = 6 * g.h2 / 32;
    g.rec_cap = p->record_cap;
    g.variant = p->variant;
    g.lpd = (p->variant & SPKMC_VARIANT_TWO_COLOURS) ? 4u : 1u;
    g.seed = p->seed;
    g.st = (DevState *)c->dev;
    g.rec = (spkmc_record *)(c->dev + lp.off_rec);
    g.Rk = (double *)(c->dev + lp.off_Rk);
    g.hist = (uint32_t *)(c->dev + lp.off_hist);
    g.flip = (uint64_t *)(c->dev + lp.off_flip);
    g.sync = (uint64_t *)(c->dev + lp.off_sync);
    g.dh = p->layout == SPKMC_LAYOUT_PACKED ? (uint64_t *)(c->dev + lp.off_dh) : nullptr;
    g.sc = p->layout == SPKMC_LAYOUT_PACKED && g.h == 16 ? (uint32_t *)(c->dev + lp.off_sc) : nullptr;
    if (p->layout == SPKMC_LAYOUT_INT8) {
        g.spin8 = (int8_t *)(c->dev + lp.off_spin);
    } else {
        g.A = (uint32_t *)(c->dev + lp.off_spin);
        g.F = (uint32_t *)(c->dev + lp.off_F);
    }
    make_rates(p, g.r);
    {   // R'_max: the sites of one line times the largest class rate
        double rb = g.r[0];
        for (int cc = 1; cc < 14; ++cc)
            if (g.r[cc] > rb) rb = g.r[cc];
        g.rbound = (double)((int64_t)g.h * g.h * g.h) * rb;
        g.pad2 = 0;
    }
    c->spin_off = lp.off_spin;
    c->spin_bytes = lp.spin_bytes;
    c->rec_off = lp.off_rec;

    // engine choice: the slab engine for an explicit request or (AUTO) the
    // all-octant R_max with domain 32; the incremental engine for an explicit
    // request or the all-octant R_max otherwise (its histograms of every octant
    // stay resident); else the re-binning persistent engine, else the per-cycle
    // engine
    std::string pwhy;
    // AUTO with the all-octant R_max: the slab engine where it runs (PACKED,
    // domain 32; it reads every octant's counts instead of keeping them on chip)
    const bool auto_slab = p->engine == SPKMC_ENGINE_AUTO && (p->variant & SPKMC_VARIANT_RMAX_ALL) &&
                           slab_supported(g, *p, pwhy) && slab_configure(g, c->grid, c->block, c->wg_domains) == hipSuccess;
    if (p->engine == SPKMC_ENGINE_SLAB || auto_slab) {
        if (!slab_supported(g, *p, pwhy)) return fail(c, SPKMC_E_UNSUPPORTED, "slab engine: " + pwhy);
        c->engine = SPKMC_ENGINE_SLAB;
        hipError_t e = slab_configure(g, c->grid, c->block, c->wg_domains);
        if (e == hipErrorCooperativeLaunchTooLarge)
            return fail(c, SPKMC_E_UNSUPPORTED, "slab engine: the domains do not fit in one resident launch");
        if (e != hipSuccess) return hip_fail(c, e, "slab_configure");
    } else {
    const bool want_inc = p->engine == SPKMC_ENGINE_INCREMENTAL ||
                          (p->engine == SPKMC_ENGINE_AUTO && (p->variant & SPKMC_VARIANT_RMAX_ALL));
    bool pers = persistent_supported(g, *p, want_inc, pwhy);
    const bool want_pers = p->engine == SPKMC_ENGINE_PERSISTENT || p->engine == SPKMC_ENGINE_INCREMENTAL;
    if (want_pers && !pers) return fail(c, SPKMC_E_UNSUPPORTED, "persistent engine: " + pwhy);
    c->engine = (p->engine == SPKMC_ENGINE_CYCLE || !pers) ? SPKMC_ENGINE_CYCLE
                : want_inc                            ? SPKMC_ENGINE_INCREMENTAL
                                                      : SPKMC_ENGINE_PERSISTENT;
    c->grid = (int)g.K;
    c->block = 256;
    c->wg_domains = 0;
    if (c->engine != SPKMC_ENGINE_CYCLE) {
        hipError_t e = persistent_configure(g, *p, c->engine == SPKMC_ENGINE_INCREMENTAL, c->grid, c->block,
                                            c->wg_domains);
        if (e == hipErrorCooperativeLaunchTooLarge && p->engine == SPKMC_ENGINE_AUTO) {
            // more domains than one resident launch holds: the per-cycle engine
            c->engine = SPKMC_ENGINE_CYCLE;
            c->grid = (int)g.K;
            c->block = 256;
            c->wg_domains = 0;
        } else if (e == hipErrorCooperativeLaunchTooLarge) {
            return fail(c, SPKMC_E_UNSUPPORTED, "persistent engine: the domains do not fit in one resident launch");
        } else if (e != hipSuccess) {
            return hip_fail(c, e, "persistent_configure");
        }
    }
    }

    hipError_t e;
    if ((e = hipMemsetAsync(c->dev, 0, lp.off_spin, c->stream)) != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
    if ((e = hipMemcpyAsync(c->dev + lp.off_rates, g.r, sizeof g.r, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "hipMemcpyAsync(rates)");
    if ((e = launch_init(g, p->init, c->stream)) != hipSuccess) return hip_fail(c, e, "init kernel");
    if ((e = launch_faces(g, c->stream)) != hipSuccess) return hip_fail(c, e, "face kernel");
    if ((e = launch_observables(g, c->stream)) != hipSuccess) return hip_fail(c, e, "observables kernel");
    return SPKMC_OK;
}

spkmc_status spkmc_run(spkmc_ctx *c, uint64_t ncycles, uint32_t obs_every) {
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (c->failed || !c->dev) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    if (ncycles == 0) return SPKMC_OK;
    hipError_t e = hipSuccess;
    if (c->engine != SPKMC_ENGINE_CYCLE) {
        // the set-up of the sync words is needed unless the previous launch left
        // them ready for this one
        const bool primed = c->primed_grid == c->grid && c->primed_cycle == c->cycle && c->primed_span >= 2;
        if (c->engine == SPKMC_ENGINE_SLAB)
            e = launch_slab(c->g, c->cycle, ncycles, obs_every, c->grid, !primed, c->stream);
        else
            e = launch_persistent(c->g, c->cycle, ncycles, obs_every, c->grid, c->block, c->wg_domains,
                                  c->engine == SPKMC_ENGINE_INCREMENTAL, !primed, c->stream);
        if (e != hipSuccess) {
            c->primed_grid = 0;
            return hip_fail(c, e, c->engine == SPKMC_ENGINE_SLAB ? "slab kernel launch" : "persistent kernel launch");
        }
        c->primed_span = (primed ? c->primed_span : 0) + ncycles;
        c->primed_grid = c->grid;
        c->cycle += ncycles;
        c->primed_cycle = c->cycle;
    } else {
        // PACKED lattices with octant edge 16 run the slab kernels, whose counts
        // are binned afresh at the start of every run
        const bool slab = slab_rows_supported(c->g);
        if (slab && (e = launch_slab_bin(c->g, c->stream)) != hipSuccess) return hip_fail(c, e, "slab count kernel");
        for (uint64_t i = 0; i < ncycles; ++i) {
            e = launch_cycle(c->g, c->cycle, obs_every, c->stream, slab);
            if (e != hipSuccess) return hip_fail(c, e, "cycle kernel launch");
            c->cycle += 1;
        }
    }
    return SPKMC_OK;
}

static spkmc_status read_state(spkmc_ctx *c, DevState &st) {
    hipError_t e = hipMemcpyAsync(&st, c->dev, sizeof st, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reading device state");
    if (st.error) {
        char m[128];
        snprintf(m, sizeof m, "device-side wait gave up (code %u)", st.error);
        return fail(c, SPKMC_E_DEVICE, m);
    }
    return SPKMC_OK;
}

spkmc_status spkmc_observables(spkmc_ctx *c, spkmc_obs *out) {
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!out) return fail(c, SPKMC_E_INVAL, "out is NULL");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    DevState st;
    spkmc_status s = read_state(c, st);
    if (s != SPKMC_OK) return s;
    obs_from_state(c->p, c->g.N, st, out);
    return SPKMC_OK;
}

spkmc_status spkmc_records(spkmc_ctx *c, spkmc_record *host, size_t cap, size_t *n) {
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!n || (!host && cap)) return fail(c, SPKMC_E_INVAL, "bad output arguments");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    DevState st;
    spkmc_status s = read_state(c, st);
    if (s != SPKMC_OK) return s;
    uint64_t have = st.rec_count < c->p.record_cap ? st.rec_count : c->p.record_cap;
    uint64_t take = have < cap ? have : cap;
    std::vector<spkmc_record> ring(c->p.record_cap ? c->p.record_cap : 1);
    if (c->p.record_cap) {
        hipError_t e = hipMemcpy(ring.data(), c->dev + c->rec_off, sizeof(spkmc_record) * c->p.record_cap, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "copying records");
    }
    for (uint64_t i = 0; i < take; ++i) {
        uint64_t idx = st.rec_count - take + i;
        host[i] = ring[idx % c->p.record_cap];
    }
    *n = (size_t)take;
    return SPKMC_OK;
}

// host-side bit address of site (x, y, z) in the packed layout
static inline uint64_t packed_bit(const Geom &g, int x, int y, int z) {
    int kx = x / g.d, ky = y / g.d, kz = z / g.d;
    int rx = x - kx * g.d, ry = y - ky * g.d, rz = z - kz * g.d;
    int sx = rx >= g.h, sy = ry >= g.h, sz = rz >= g.h;
    uint64_t k = (uint64_t)kx + (uint64_t)g.nd * ((uint64_t)ky + (uint64_t)g.nd * (uint64_t)kz);
    uint64_t q = (uint64_t)(rx - sx * g.h) + (uint64_t)g.h * ((uint64_t)(ry - sy * g.h) + (uint64_t)g.h * (uint64_t)(rz - sz * g.h));
    return (k * 8 + (uint64_t)(sx | (sy << 1) | (sz << 2))) * g.h3 + q;
}

spkmc_status spkmc_copy_spins(spkmc_ctx *c, int8_t *host, size_t n) {
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!host) return fail(c, SPKMC_E_INVAL, "host is NULL");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    if (n < c->g.N) return fail(c, SPKMC_E_RANGE, "host buffer smaller than N");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    const Geom &g = c->g;
    if (g.layout == SPKMC_LAYOUT_INT8) {
        e = hipMemcpy(host, c->dev + c->spin_off, g.N, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "copying spins");
        return SPKMC_OK;
    }
    std::vector<uint32_t> A;
    try {
        A.resize(g.N / 32);
    } catch (...) {
        return fail(c, SPKMC_E_NOMEM, "host buffer for packed spins");
    }
    e = hipMemcpy(A.data(), c->dev + c->spin_off, g.N / 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "copying spins");
    // octant-major -> linear
    for (uint64_t o = 0; o < (uint64_t)g.K * 8; ++o) {
        uint32_t k = (uint32_t)(o >> 3);
        int s = (int)(o & 7);
        int kx = (int)(k % (uint32_t)g.nd), ky = (int)((k / (uint32_t)g.nd) % (uint32_t)g.nd), kz = (int)(k / ((uint32_t)g.nd * (uint32_t)g.nd));
        int ox = kx * g.d + (s & 1) * g.h, oy = ky * g.d + ((s >> 1) & 1) * g.h, oz = kz * g.d + ((s >> 2) & 1) * g.h;
        const uint32_t *w = &A[o * g.wpo];
        uint32_t q = 0;
        for (int lz = 0; lz < g.h; ++lz)
            for (int ly = 0; ly < g.h; ++ly) {
                int8_t *row = host + (uint64_t)ox + (uint64_t)g.L * ((uint64_t)(oy + ly) + (uint64_t)g.L * (uint64_t)(oz + lz));
                for (int lx = 0; lx < g.h; ++lx, ++q) row[lx] = ((w[q >> 5] >> (q & 31)) & 1u) ? 1 : -1;
            }
    }
    return SPKMC_OK;
}

static void host_observables(const int8_t *s, int L, int64_t &M, int64_t &B) {
    M = 0;
    B = 0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int v = s[(int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * z)];
                M += v;
                B += v * (s[(int64_t)(x + 1 == L ? 0 : x + 1) + (int64_t)L * ((int64_t)y + (int64_t)L * z)] +
                          s[(int64_t)x + (int64_t)L * ((int64_t)(y + 1 == L ? 0 : y + 1) + (int64_t)L * z)] +
                          s[(int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * (z + 1 == L ? 0 : z + 1))]);
            }
}

spkmc_status spkmc_set_spins(spkmc_ctx *c, const int8_t *host, size_t n) {
    if (c) c->primed_grid = 0;
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!host) return fail(c, SPKMC_E_INVAL, "host is NULL");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    const Geom &g = c->g;
    if (n < g.N) return fail(c, SPKMC_E_RANGE, "host buffer smaller than N");
    for (uint64_t i = 0; i < g.N; ++i)
        if (host[i] != 1 && host[i] != -1) return fail(c, SPKMC_E_INVAL, "spins must be +1 or -1");
    int64_t M, B;
    host_observables(host, g.L, M, B);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    if (g.layout == SPKMC_LAYOUT_INT8) {
        e = hipMemcpy(c->dev + c->spin_off, host, g.N, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "copying spins");
    } else {
        std::vector<uint32_t> A(g.N / 32, 0u);
        for (int z = 0; z < g.L; ++z)
            for (int y = 0; y < g.L; ++y)
                for (int x = 0; x < g.L; ++x)
                    if (host[(int64_t)x + (int64_t)g.L * ((int64_t)y + (int64_t)g.L * z)] > 0) {
                        uint64_t b = packed_bit(g, x, y, z);
                        A[b >> 5] |= 1u << (b & 31);
                    }
        e = hipMemcpy(c->dev + c->spin_off, A.data(), g.N / 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "copying spins");
        if ((e = launch_faces(g, c->stream)) != hipSuccess) return hip_fail(c, e, "face kernel");
    }
    DevState st;
    e = hipMemcpy(&st, c->dev, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "reading state");
    st.M = M;
    st.B = B;
    e = hipMemcpy(c->dev, &st, sizeof st, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "writing state");
    return SPKMC_OK;
}

static const uint64_t kMagic = 0x31434d4b50535053ull;  // "SPSPKMC1"

spkmc_status spkmc_save(spkmc_ctx *c, void *host, size_t cap, size_t *n) {
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!n) return fail(c, SPKMC_E_INVAL, "n is NULL");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    size_t need = 8 + sizeof(spkmc_params) + 8 + c->spin_off + c->spin_bytes;
    *n = need;
    if (!host) return SPKMC_OK;
    if (cap < need) return fail(c, SPKMC_E_RANGE, "checkpoint buffer too small");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    char *o = (char *)host;
    memcpy(o, &kMagic, 8);
    memcpy(o + 8, &c->p, sizeof(spkmc_params));
    memcpy(o + 8 + sizeof(spkmc_params), &c->cycle, 8);
    // DevState, rates, records, per-domain scratch and spins, as laid out on the device
    e = hipMemcpy(o + 16 + sizeof(spkmc_params), c->dev, c->spin_off + c->spin_bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "copying state");
    return SPKMC_OK;
}

spkmc_status spkmc_load(spkmc_ctx *c, const void *host, size_t n) {
    if (c) c->primed_grid = 0;
    if (!c) return fail(nullptr, SPKMC_E_INVAL, "ctx is NULL");
    if (!host) return fail(c, SPKMC_E_INVAL, "host is NULL");
    if (c->failed) return fail(c, SPKMC_E_STATE, "context is in a failed state");
    size_t need = 8 + sizeof(spkmc_params) + 8 + c->spin_off + c->spin_bytes;
    if (n != need) return fail(c, SPKMC_E_INVAL, "checkpoint size does not match these parameters");
    const char *o = (const char *)host;
    uint64_t magic;
    memcpy(&magic, o, 8);
    if (magic != kMagic) return fail(c, SPKMC_E_INVAL, "not a checkpoint");
    spkmc_params p;
    memcpy(&p, o + 8, sizeof p);
    // the initial-state choice and the launch shape do not change the meaning of a saved state
    p.init = c->p.init;
    p.engine = c->p.engine;
    p.wg_domains = c->p.wg_domains;
    if (memcmp(&p, &c->p, sizeof p) != 0) return fail(c, SPKMC_E_INVAL, "checkpoint parameters differ");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    e = hipMemcpy(c->dev, o + 16 + sizeof(spkmc_params), c->spin_off + c->spin_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "copying state");
    memcpy(&c->cycle, o + 8 + sizeof(spkmc_params), 8);
    return SPKMC_OK;
}

spkmc_status spkmc_query(const spkmc_ctx *c, spkmc_info *out) {
    if (!c || !out) return fail(nullptr, SPKMC_E_INVAL, "NULL argument");
    out->engine = c->engine;
    out->layout = c->g.layout;
    out->h = c->g.h;
    out->grid = c->grid;
    out->block = c->block;
    out->wg_domains = c->wg_domains;
    out->K = c->g.K;
    out->N = c->g.N;
    out->state_bytes = c->spin_off + c->spin_bytes;
    double h = c->g.h;
    // every frequency line (an active octant: one per domain, four with two colours)
    out->bytes_per_cycle = (double)c->g.K * c->g.lpd * ((h * h * h + 6.0 * h * h) / 8.0 + 8.0);
    // slab engine: the active octant's 28 count words are read and written back too
    if (c->engine == SPKMC_ENGINE_SLAB) out->bytes_per_cycle += (double)c->g.K * 2.0 * 28.0 * 4.0;
    return SPKMC_OK;
}

size_t spkmc_batch_workspace_bytes(size_t n) { return align256(n * replica_bytes()); }

}  // extern "C"

// A batch, checked and planned: its members with work, their cycle counts, the
// host descriptors and the launch shape.
struct BatchPlan {
    std::vector<spkmc_ctx *> live;
    std::vector<uint64_t> nc;
    std::vector<unsigned char> host;  // the descriptors (replica_bytes() each)
    hipStream_t stream = nullptr;
    int h = 0, grid = 0, block = 0, P = 0;
    uint32_t lpd = 1;  // every lattice with one line per domain (else 0)
};

static spkmc_status plan_batch(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                               int32_t wg_domains, void *dev_workspace, size_t ws_bytes, BatchPlan &bp) {
    if (!ctxs || !ncycles || n == 0) return fail(nullptr, SPKMC_E_INVAL, "no lattices");
    if (!dev_workspace || ws_bytes < spkmc_batch_workspace_bytes(n))
        return fail(nullptr, SPKMC_E_RANGE, "batch workspace too small");
    std::vector<const Geom *> gs;
    std::vector<uint64_t> n0;
    for (size_t i = 0; i < n; ++i) {
        spkmc_ctx *c = ctxs[i];
        if (!c) return fail(nullptr, SPKMC_E_INVAL, "NULL context in batch");
        if (c->failed || !c->dev) return fail(nullptr, SPKMC_E_STATE, "a context of the batch is in a failed state");
        if (ncycles[i] == 0) continue;
        if (std::find(bp.live.begin(), bp.live.end(), c) != bp.live.end())
            return fail(nullptr, SPKMC_E_INVAL, "a context appears twice in the batch");
        std::string why;
        if (!persistent_supported(c->g, c->p, false, why)) return fail(nullptr, SPKMC_E_UNSUPPORTED, "batch member: " + why);
        if (bp.live.empty()) {
            bp.stream = c->stream;
            bp.h = c->g.h;
        } else if (c->stream != bp.stream || c->g.h != bp.h) {
            return fail(nullptr, SPKMC_E_INVAL, "batch members must share the stream and the octant edge");
        }
        bp.live.push_back(c);
        gs.push_back(&c->g);
        n0.push_back(c->cycle);
        bp.nc.push_back(ncycles[i]);
    }
    if (bp.live.empty()) return SPKMC_OK;
    const int rows = persist_rows(bp.h, false), pmax = batch_max_passes(bp.h);
    std::vector<int> Ps;
    if (wg_domains) {
        const int pc = wg_domains / rows;
        if (wg_domains % rows || pc > pmax || (pc & (pc - 1)))
            return fail(nullptr, SPKMC_E_INVAL, "wg_domains must be 1, 2 or 4 passes of the row count (at most " +
                                                    std::to_string(pmax) + " for this octant edge)");
        Ps.push_back(pc);
    } else {
        for (int P = 1; P <= pmax; P <<= 1) Ps.push_back(P);
    }
    bp.host.resize(replica_bytes() * bp.live.size());
    Replica *reps = reinterpret_cast<Replica *>(bp.host.data());
    hipError_t e = hipErrorCooperativeLaunchTooLarge;
    for (int Pc : Ps) {
        e = batch_plan(gs.data(), n0.data(), bp.nc.data(), obs_every, (uint32_t)bp.live.size(), Pc, reps, bp.grid,
                       bp.block, bp.lpd);
        if (e == hipSuccess) {
            bp.P = Pc;
            break;
        }
    }
    if (e == hipErrorCooperativeLaunchTooLarge)
        return fail(nullptr, SPKMC_E_UNSUPPORTED, "the batch does not fit on the device at once: split it");
    if (e != hipSuccess) return fail(nullptr, SPKMC_E_DEVICE, std::string("batch plan: ") + hipGetErrorString(e));
    return SPKMC_OK;
}

static void batch_info_of(const BatchPlan &bp, spkmc_batch_info *info) {
    if (!info) return;
    uint64_t domains = 0;
    for (spkmc_ctx *c : bp.live) domains += c->g.K;
    info->grid = bp.grid;
    info->block = bp.block;
    info->wg_domains = (bp.block / 16) * bp.P;
    info->h = bp.h;
    info->lattices = bp.live.size();
    info->domains = domains;
}

struct spkmc_batch_graph {
    std::vector<spkmc_ctx *> members;
    std::vector<uint64_t> nc;      // cycles per replay
    std::vector<uint64_t> expect;  // each member's cycle count when the next replay starts
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

}  // extern "C"

// Upload a planned batch's descriptors to dev_reps and launch it.
static spkmc_status launch_planned(BatchPlan &bp, Replica *dev_reps, spkmc_batch_info *info) {
    const uint32_t nl = (uint32_t)bp.live.size();
    hipError_t e = upload_replicas(reinterpret_cast<const Replica *>(bp.host.data()), nl, dev_reps, bp.stream);
    if (e == hipSuccess) e = launch_batch(dev_reps, nl, bp.h, bp.P, bp.grid, bp.block, bp.lpd, bp.stream);
    if (e != hipSuccess) {
        for (spkmc_ctx *c : bp.live) c->failed = true;
        return fail(nullptr, SPKMC_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    }
    for (size_t i = 0; i < bp.live.size(); ++i) {
        bp.live[i]->cycle += bp.nc[i];
        bp.live[i]->primed_grid = 0;  // a batch lays out the sync words for its own grid
    }
    batch_info_of(bp, info);
    return SPKMC_OK;
}

extern "C" {

spkmc_status spkmc_run_batch(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                             int32_t wg_domains, void *dev_workspace, size_t ws_bytes, spkmc_batch_info *info) {
    BatchPlan bp;
    spkmc_status st = plan_batch(ctxs, n, ncycles, obs_every, wg_domains, dev_workspace, ws_bytes, bp);
    if (st != SPKMC_OK || bp.live.empty()) return st;
    return launch_planned(bp, reinterpret_cast<Replica *>(dev_workspace), info);
}

spkmc_status spkmc_run_batch_static(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                                    int32_t wg_domains, spkmc_batch_info *info) {
    if (n > static_replica_cap())
        return fail(nullptr, SPKMC_E_RANGE,
                    "spkmc_run_batch_static takes at most " + std::to_string(static_replica_cap()) + " lattices");
    Replica *dev_reps = nullptr;
    hipError_t e = static_replicas(&dev_reps);
    if (e != hipSuccess)
        return fail(nullptr, SPKMC_E_DEVICE, std::string("static descriptor array: ") + hipGetErrorString(e));
    BatchPlan bp;
    spkmc_status st = plan_batch(ctxs, n, ncycles, obs_every, wg_domains, dev_reps, static_replica_bytes(), bp);
    if (st != SPKMC_OK || bp.live.empty()) return st;
    return launch_planned(bp, dev_reps, info);
}

spkmc_status spkmc_batch_graph_create(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                                      int32_t wg_domains, void *dev_workspace, size_t ws_bytes,
                                      spkmc_batch_info *info, spkmc_batch_graph **out) {
    if (!out) return fail(nullptr, SPKMC_E_INVAL, "out is NULL");
    *out = nullptr;
    BatchPlan bp;
    spkmc_status st = plan_batch(ctxs, n, ncycles, obs_every, wg_domains, dev_workspace, ws_bytes, bp);
    if (st != SPKMC_OK) return st;
    if (bp.live.empty()) return fail(nullptr, SPKMC_E_INVAL, "no lattice of the batch has cycles to run");
    const uint32_t nl = (uint32_t)bp.live.size();
    Replica *dev_reps = reinterpret_cast<Replica *>(dev_workspace);
    hipError_t e = upload_replicas(reinterpret_cast<const Replica *>(bp.host.data()), nl, dev_reps, bp.stream);
    if (e != hipSuccess) return fail(nullptr, SPKMC_E_DEVICE, std::string("batch upload: ") + hipGetErrorString(e));
    auto *gr = new spkmc_batch_graph;
    gr->members = bp.live;
    gr->nc = bp.nc;
    gr->stream = bp.stream;
    for (spkmc_ctx *c : bp.live) {
        gr->expect.push_back(c->cycle);
        c->primed_grid = 0;
    }
    e = capture_batch(dev_reps, nl, bp.h, bp.P, bp.grid, bp.block, bp.lpd, &gr->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        spkmc_batch_graph_destroy(gr);
        (void)hipGetLastError();
        return fail(nullptr, SPKMC_E_UNSUPPORTED, std::string("batch graph: ") + hipGetErrorString(e));
    }
    batch_info_of(bp, info);
    *out = gr;
    return SPKMC_OK;
}

spkmc_status spkmc_batch_graph_launch(spkmc_batch_graph *gr, uint32_t replays) {
    if (!gr || !gr->exec) return fail(nullptr, SPKMC_E_INVAL, "graph is NULL");
    for (size_t i = 0; i < gr->members.size(); ++i) {
        spkmc_ctx *c = gr->members[i];
        if (c->failed) return fail(nullptr, SPKMC_E_STATE, "a member of the graph is in a failed state");
        if (c->cycle != gr->expect[i])
            return fail(nullptr, SPKMC_E_STATE, "a member of the graph was advanced outside the graph");
    }
    for (uint32_t r = 0; r < replays; ++r) {
        hipError_t e = hipGraphLaunch(gr->exec, gr->stream);
        if (e != hipSuccess) {
            for (spkmc_ctx *c : gr->members) c->failed = true;
            return fail(nullptr, SPKMC_E_DEVICE, std::string("batch graph launch: ") + hipGetErrorString(e));
        }
        for (size_t i = 0; i < gr->members.size(); ++i) {
            gr->members[i]->cycle += gr->nc[i];
            gr->expect[i] += gr->nc[i];
        }
    }
    return SPKMC_OK;
}

void spkmc_batch_graph_destroy(spkmc_batch_graph *gr) {
    if (!gr) return;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
}

const char *spkmc_last_error(const spkmc_ctx *c) {
    if (c) return c->err.empty() ? "no error" : c->err.c_str();
    return g_last_error.c_str();
}

void spkmc_destroy(spkmc_ctx *c) { delete c; }

}  // extern "C"
#pragma GCC visibility pop
