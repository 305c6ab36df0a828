// rt_host.cpp -- C ABI of the renderer: argument validation, the
// channel-independent constants of the line (in double, once per call), the
// partition-function table, and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rtcube.h"
#include "rt_host.h"
#include "rt_kernels.h"
#include "rt_launch.h"

namespace rt {

// cgs constants (CODATA 2018), typed here on their own
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kC = 2.99792458e10;
constexpr double kAMU = 1.66053906660e-24;
constexpr double kAU = 1.495978707e13;
constexpr double kPI = 3.14159265358979323846;

static thread_local std::string g_err;

rt_status fail(rt_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rt_status fail_hip(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- options
static int64_t g_opt_cb = 0;
static int64_t g_opt_thin = 1;
static int64_t g_opt_ckpt = 0;
static int64_t g_opt_split = 0;
static int64_t g_opt_accum = 0;
static int64_t g_opt_adj_cap = 0;
static int64_t g_opt_adj_cb = 0;
static int64_t g_opt_adj_lanes = 0;
static int64_t g_opt_group = 0;

// Launch shape of the forward march: channels per lane (cb) and lanes per
// ray (nsplit).  Measured on MI355X: one channel block per pixel is best
// (the shading is not repeated), and a launch needs about 4096 waves (4 per
// SIMD) before it stops losing time to latency and to its last partial round
// of waves; so take the smallest block holding all channels (at most 64),
// then split rays until the launch has 4096 waves.  64-channel blocks split
// into 32-channel blocks instead (their registers no longer fit two lanes'
// worth of live ray state), and 48-channel blocks split at most 4 ways.
void forward_shape(int nch, long npix, int nsamp, int *cb_out, int *split_out) {
    static const int cands[] = {8, 16, 24, 32, 48, 64};
    int cb = 64;
    for (int c : cands)
        if (c >= nch) { cb = c; break; }
    if (g_opt_cb) cb = (int)g_opt_cb;
    auto waves = [&](int c, int ns) { return ((npix * ns + 63) / 64) * (long)((nch + c - 1) / c); };
    if (!g_opt_cb && cb == 64 && waves(64, 1) < 4096) cb = 32;
    const int max_split = cb >= 64 ? 1 : (cb >= 48 ? 4 : 8);
    int ns = 1;
    while (ns < max_split && waves(cb, ns) < 4096 && nsamp >= 32 * ns) ns <<= 1;
    *cb_out = cb;
    *split_out = ns;
}

int channel_block_for(int nch, long npix) {
    int cb, ns;
    forward_shape(nch, npix, 1 << 20, &cb, &ns);
    return cb;
}

bool thin_series() { return g_opt_thin != 0; }
int ckpt_segment_option() { return (int)g_opt_ckpt; }
int ray_split_option() { return (int)g_opt_split; }
int channel_block_option() { return (int)g_opt_cb; }
bool grad_accum_double() { return g_opt_accum != 0; }
int adjoint_block_option() { return (int)g_opt_adj_cb; }
int adjoint_lanes_option() { return (int)g_opt_adj_lanes; }
size_t adjoint_scratch_cap() { return g_opt_adj_cap > 0 ? (size_t)g_opt_adj_cap : kAdjointScratchCap; }

// ---------------------------------------------------------------- validation
static bool finite(double x) { return std::isfinite(x); }

// line, camera, spectral axis and sampling, shared by every renderer
rt_status validate_view(const rt_line &l, const rt_camera &c, const rt_spectral &s, int32_t nsamp,
                        double intensity_scale, double max_incl_deg) {
    if (!(finite(l.nu0_hz) && l.nu0_hz > 0 && finite(l.a_ul) && l.a_ul >= 0 && l.g_u > 0 && l.g_l > 0 &&
          finite(l.g_u) && finite(l.g_l) && finite(l.e_u_k) && finite(l.e_l_k) && l.e_l_k >= 0 &&
          l.m_co_amu > 0 && l.m_mol_amu > 0 && finite(l.m_co_amu) && finite(l.m_mol_amu)))
        return fail(RT_EINVAL, "invalid line data");
    if (l.nlev < 1 || !l.lev_e_k || !l.lev_g) return fail(RT_EINVAL, "level table missing");
    for (int i = 0; i < l.nlev; ++i)
        if (!(finite(l.lev_e_k[i]) && l.lev_e_k[i] >= 0 && finite(l.lev_g[i]) && l.lev_g[i] >= 0))
            return fail(RT_EINVAL, "invalid level %d", i);
    if (c.nx < 1 || c.ny < 1) return fail(RT_EINVAL, "need nx, ny >= 1");
    if ((int64_t)c.nx * c.ny > (int64_t)1 << 30) return fail(RT_EINVAL, "image too large");
    if (!(finite(c.fov_au) && c.fov_au > 0)) return fail(RT_EINVAL, "need fov_au > 0");
    if (!(finite(c.incl_deg) && c.incl_deg >= 0 && c.incl_deg <= max_incl_deg))
        return fail(RT_EINVAL, "inclination must be within [0, %g] deg", max_incl_deg);
    if (!finite(c.pa_deg)) return fail(RT_EINVAL, "position angle not finite");
    if (s.nch < 1 || s.nch > RT_MAX_CHANNELS) return fail(RT_EINVAL, "need 1 <= nch <= %d", RT_MAX_CHANNELS);
    if (!s.v_kms) return fail(RT_EINVAL, "channel velocities missing");
    for (int i = 0; i < s.nch; ++i)
        if (!finite(s.v_kms[i])) return fail(RT_EINVAL, "channel %d velocity not finite", i);
    if (!finite(s.v_sys_kms)) return fail(RT_EINVAL, "v_sys not finite");
    if (nsamp < 1 || nsamp > (1 << 20)) return fail(RT_EINVAL, "need 1 <= nsamp <= 2^20");
    if (!finite(intensity_scale)) return fail(RT_EINVAL, "intensity_scale not finite");
    return RT_OK;
}

rt_status validate(const rt_problem *p) {
    if (!p) return fail(RT_EINVAL, "problem is NULL");
    const rt_grid &g = p->grid;
    if (g.nr < 2 || g.nz < 2) return fail(RT_EINVAL, "grid needs nr >= 2 and nz >= 2 (got %d, %d)", g.nr, g.nz);
    if ((int64_t)g.nr * g.nz > (int64_t)1 << 30) return fail(RT_EINVAL, "grid too large");
    if (!(finite(g.r_min_au) && finite(g.r_max_au) && g.r_min_au > 0 && g.r_max_au > g.r_min_au))
        return fail(RT_EINVAL, "need 0 < r_min_au < r_max_au");
    if (!(finite(g.zr_max) && g.zr_max > 0)) return fail(RT_EINVAL, "need zr_max > 0");
    const rt_fields &f = p->f;
    if (!f.ln_nh2 || !f.temp_k || !f.vphi_kms || !f.z_lo_au || !f.z_up_au)
        return fail(RT_EINVAL, "a field pointer is NULL");
    if (!(finite(f.x_co) && f.x_co >= 0)) return fail(RT_EINVAL, "need x_co >= 0");
    if (!(finite(f.mask_width) && f.mask_width > 0)) return fail(RT_EINVAL, "need mask_width > 0");
    if (!(finite(f.v_turb) && f.v_turb >= 0)) return fail(RT_EINVAL, "need v_turb >= 0");
    rt_status st = validate_view(p->line, p->cam, p->spec, p->nsamp, p->intensity_scale, 90.0);
    if (st != RT_OK) return st;
    if (p->mlp) {
        if (!p->mlp->weights) return fail(RT_EINVAL, "mlp weights missing");
        if (p->mlp->precision != RT_MLP_FP32 && p->mlp->precision != RT_MLP_BF16)
            return fail(RT_EINVAL, "unknown mlp precision %d", p->mlp->precision);
    }
    return RT_OK;
}

// ---------------------------------------------------------------- Z(T) table
struct ZKey {
    int dev;
    uint64_t hash;
    bool operator<(const ZKey &o) const { return dev != o.dev ? dev < o.dev : hash < o.hash; }
};
static std::mutex g_ztab_mu;
static std::map<ZKey, float4 *> g_ztab;

static uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

constexpr double kZT0 = 0.1, kZT1 = 1.0e4;

// The adjoint and network scratch (up to tens of GB) comes from the
// device's default stream-ordered pool; keep freed blocks in the pool rather
// than unmapping them at every synchronisation, so repeated calls reuse them.
void trim_memory_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
}

static void keep_pool(int dev) {
    static std::mutex mu;
    static std::map<int, bool> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev]) return;
    done[dev] = true;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
}

namespace {
struct WsKey {
    int dev;
    hipStream_t st;
    int slot;
    bool operator<(const WsKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (st != o.st) return st < o.st;
        return slot < o.slot;
    }
};
struct WsBuf {
    void *p = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<WsKey, WsBuf> g_ws;
} // namespace

// workspaces grow in 64 MiB steps
size_t workspace_round(size_t bytes) { return (bytes + (64u << 20) - 1) / (64u << 20) * (64u << 20); }

void *stream_workspace(hipStream_t st, int slot, size_t bytes, hipError_t *err) {
    *err = hipSuccess;
    int dev = 0;
    if ((*err = hipGetDevice(&dev)) != hipSuccess) return nullptr;
    keep_pool(dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsBuf &b = g_ws[{dev, st, slot}];
    if (b.bytes >= bytes && b.p) return b.p;
    // the old buffer is released in stream order, after the work already
    // queued on this stream that may still use it
    const size_t want = workspace_round(bytes);
    if (b.p) {
        if ((*err = hipFreeAsync(b.p, st)) != hipSuccess) return nullptr;
        b.p = nullptr;
        b.bytes = 0;
    }
    if ((*err = hipMallocAsync(&b.p, want, st)) != hipSuccess) {
        // the error goes back to the caller; it must not linger as this
        // thread's last error and fail a later launch check
        (void)hipGetLastError();
        b.p = nullptr;
        return nullptr;
    }
    b.bytes = want;
    return b.p;
}

size_t stream_workspace_bytes(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    size_t n = 0;
    for (const auto &kv : g_ws)
        if (kv.first.st == st) n += kv.second.bytes;
    return n;
}

void release_stream_workspaces(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.st == st) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(it->first.dev);
            (void)hipFreeAsync(it->second.p, st);
            (void)hipSetDevice(cur);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
}

void partition_table_host(const rt_line &l, float4 *tab) {
    const int N = kZTableNodes;
    const double l0 = std::log2(kZT0), l1 = std::log2(kZT1), step = (l1 - l0) / (N - 1);
    std::vector<double> z(N), dz(N);
    for (int i = 0; i < N; ++i) {
        const double T = std::exp2(l0 + i * step);
        double s = 0.0, d = 0.0;
        for (int j = 0; j < l.nlev; ++j) {
            const double w = l.lev_g[j] * std::exp(-l.lev_e_k[j] / T);
            s += w;
            d += w * l.lev_e_k[j] / T;
        }
        z[i] = s;
        dz[i] = d * std::log(2.0) * step;   // dZ/d(table index)
    }
    for (int i = 0; i < N - 1; ++i)
        tab[i] = make_float4((float)z[i], (float)dz[i], (float)z[i + 1], (float)dz[i + 1]);
}

rt_status partition_table(const rt_line &l, const float4 **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    keep_pool(dev);
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &l.nlev, sizeof l.nlev);
    h = fnv(h, l.lev_e_k, sizeof(double) * l.nlev);
    h = fnv(h, l.lev_g, sizeof(double) * l.nlev);
    std::lock_guard<std::mutex> lk(g_ztab_mu);
    auto it = g_ztab.find({dev, h});
    if (it != g_ztab.end()) { *out = it->second; return RT_OK; }
    const int N = kZTableNodes;
    std::vector<float4> tab(N - 1);
    partition_table_host(l, tab.data());
    float4 *d = nullptr;
    e = hipMalloc(&d, sizeof(float4) * (N - 1));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(partition table)");
    e = hipMemcpy(d, tab.data(), sizeof(float4) * (N - 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(d); return fail_hip(e, "hipMemcpy(partition table)"); }
    g_ztab[{dev, h}] = d;
    *out = d;
    return RT_OK;
}

// ---------------------------------------------------------------- set-up
rt_status build_launch(const rt_problem *p, Geometry *g, Shade *s, const float4 *ztab) {
    const rt_grid &gr = p->grid;
    const double dln = std::log(gr.r_max_au / gr.r_min_au) / (gr.nr - 1);
    const double dzr = gr.zr_max / (gr.nz - 1);
    const double ang = p->cam.incl_deg * kPI / 180.0, pa = p->cam.pa_deg * kPI / 180.0;
    std::memset(g, 0, sizeof *g);
    g->d_pix = p->cam.fov_au / p->cam.nx;
    g->cpa = std::cos(pa);
    g->spa = std::sin(pa);
    g->si = std::sin(ang);
    g->ci = std::cos(ang);
    if (p->cam.incl_deg == 0.0) { g->si = 0.0; g->ci = 1.0; }
    if (p->cam.incl_deg == 90.0) { g->si = 1.0; g->ci = 0.0; }
    g->rc = gr.r_max_au * std::exp(dln);
    g->zc = (gr.zr_max + dzr) * g->rc;
    g->nx = p->cam.nx;
    g->ny = p->cam.ny;
    g->xc = 0.5 * p->cam.nx;
    g->yc = 0.5 * p->cam.ny;
    g->nsamp = p->nsamp;

    std::memset(s, 0, sizeof *s);
    const rt_line &l = p->line;
    const float4 *tab = ztab;
    if (!tab) {
        rt_status st = partition_table(l, &tab);
        if (st != RT_OK) return st;
    }
    s->ln_n = p->f.ln_nh2;
    s->temp = p->f.temp_k;
    s->vphi = p->f.vphi_kms;
    s->zlo = p->f.z_lo_au;
    s->zup = p->f.z_up_au;
    s->ztab = tab;
    s->nr = gr.nr;
    s->nz = gr.nz;
    s->u_scale = (float)(std::log(2.0) / dln);
    s->log2_rmin = (float)std::log2(gr.r_min_au);
    s->inv_dzr = (float)(1.0 / dzr);
    s->fnr = (float)gr.nr;
    s->fnz = (float)gr.nz;
    const double log2e = 1.0 / std::log(2.0);
    s->inv_w = (float)(log2e / (p->f.mask_width * dzr));
    const double l0 = std::log2(kZT0), l1 = std::log2(kZT1);
    s->zt_l2t0 = (float)l0;
    s->zt_scale = (float)((kZTableNodes - 1) / (l1 - l0));
    s->el_log2e = (float)(l.e_l_k * log2e);
    const double nu = l.nu0_hz;
    s->theta = (float)(kH * nu / kKB);
    s->c_s = (float)(p->intensity_scale * 2.0 * kH * nu * nu * nu / (kC * kC));
    const double bul = l.a_ul * kC * kC / (2.0 * kH * nu * nu * nu);
    const double blu = l.g_u / l.g_l * bul;
    s->c_k = (float)(p->f.x_co * (kH * nu / (4.0 * kPI)) * blu * l.g_l * (kC / nu) * kAU /
                     (std::sqrt(kPI) * 1e5) * log2e);
    s->c_alpha = (float)((2.0 * kKB / (l.m_co_amu * kAMU) +
                          p->f.v_turb * p->f.v_turb * 2.0 * kKB / (l.m_mol_amu * kAMU)) / 1e10);
    s->sqrt_log2e = (float)std::sqrt(log2e);
    s->vrot = (float)g->si;
    s->vsys = (float)p->spec.v_sys_kms;
    s->zr_max = (float)gr.zr_max;
    s->mlp_o = nullptr;
    s->o_plane = (int64_t)p->cam.nx * p->cam.ny;
    s->o_pix0 = 0;
    return RT_OK;
}

// Marches with G lanes per pixel of cb channels each need, in every block
// of G cb channels, the velocities of lane m's channels (c + m cb) to be lane
// 0's plus m shift (uniform spacing gives shift = cb dv).  True, with the
// shift, if the n velocities v[] allow it (to 1e-9 of the velocity span: the
// float velocities the kernels use round far coarser).
bool group_shift(const double *v, int n, int G, int cb, double *shift) {
    if (n <= cb) { *shift = 0.0; return true; }
    const double sh = v[cb] - v[0];
    double span = 0.0;
    for (int c = 0; c < n; ++c) span = std::max(span, std::fabs(v[c] - v[0]));
    const double tol = 1e-9 * std::max(span, 1e-12);
    for (int b = 0; b < n; b += G * cb)
        for (int m = 1; m < G; ++m)
            for (int c = b; c < b + cb && c + m * cb < n; ++c)
                if (std::fabs(v[c + m * cb] - v[c] - m * sh) > tol) return false;
    *shift = sh;
    return true;
}

// lanes per pixel of the forward march of 64-channel blocks.  Measured on
// MI355X (512^2 x 64 x 512, disks 2000-2005): 2 lanes (104 VGPRs, 4 waves
// per SIMD) 3-7 % and 4 lanes (67 VGPRs, 7 waves) 16-18 % faster than one.
static int forward_group() { return g_opt_group ? (int)g_opt_group : 4; }

// Forward march of the whole cube, one launch per chunk of channels.
rt_status march_cube(const rt_problem *p, const Geometry &g, const Shade &s, float *cube, hipStream_t stream) {
    int cb, nsplit;
    forward_shape(std::min(p->spec.nch, kLaunchChannels), (long)p->cam.nx * p->cam.ny, p->nsamp, &cb, &nsplit);
    if (g_opt_split) nsplit = (int)g_opt_split;
    const size_t plane = (size_t)p->cam.nx * p->cam.ny;
    for (int c0 = 0; c0 < p->spec.nch; c0 += kLaunchChannels) {
        Channels ch;
        std::memset(&ch, 0, sizeof ch);
        ch.n = std::min(kLaunchChannels, p->spec.nch - c0);
        for (int c = 0; c < ch.n; ++c) ch.v[c] = (float)p->spec.v_kms[c0 + c];
        double shift = 0.0;
        hipError_t e;
        const int G = forward_group();
        if (cb == 64 && nsplit == 1 && G > 1 && group_shift(p->spec.v_kms + c0, ch.n, G, 64 / G, &shift))
            e = launch_forward_group(g, s, ch, cube + (size_t)c0 * plane, thin_series(), G, (float)shift, stream);
        else
            e = launch_forward(g, s, ch, cube + (size_t)c0 * plane, cb, thin_series(), nsplit, stream);
        if (e != hipSuccess) return fail_hip(e, "forward launch");
    }
    return RT_OK;
}

} // namespace rt

using namespace rt;

extern "C" {

const char *rt_last_error(void) { return g_err.c_str(); }
int32_t rt_abi_version(void) { return RT_ABI_VERSION; }

int32_t rt_constants(double *out, int32_t n) {
    const double v[6] = {kH, kKB, kC, kAMU, kAU, kPI};
    for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
    return 6;
}

rt_status rt_set_option(int32_t key, int64_t value) {
    switch (key) {
    case RT_OPT_CHANNEL_BLOCK:
        if (value != 0 && value != 8 && value != 16 && value != 24 && value != 32 && value != 48 && value != 64)
            return fail(RT_EINVAL, "channel block must be 0, 8, 16, 24, 32, 48 or 64");
        g_opt_cb = value;
        return RT_OK;
    case RT_OPT_THIN_EXPM1:
        g_opt_thin = value ? 1 : 0;
        return RT_OK;
    case RT_OPT_CKPT_SEGMENT:
        if (value < 0 || value > 64) return fail(RT_EINVAL, "checkpoint segment must be 0..64");
        g_opt_ckpt = value;
        return RT_OK;
    case RT_OPT_GRAD_ACCUM:
        g_opt_accum = value ? 1 : 0;
        return RT_OK;
    case RT_OPT_ADJ_SCRATCH_CAP:
        if (value < 0) return fail(RT_EINVAL, "scratch cap must be >= 0");
        g_opt_adj_cap = value;
        return RT_OK;
    case RT_OPT_ADJ_CHANNEL_BLOCK:
        if (value != 0 && value != 8 && value != 16 && value != 24 && value != 25 && value != 32)
            return fail(RT_EINVAL, "adjoint channel block must be 0, 8, 16, 24, 25 or 32");
        g_opt_adj_cb = value;
        return RT_OK;
    case RT_OPT_ADJ_PIXEL_LANES:
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return fail(RT_EINVAL, "adjoint lanes per pixel must be 0, 1, 2 or 4");
        g_opt_adj_lanes = value;
        return RT_OK;
    case RT_OPT_RAY_SPLIT:
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
            return fail(RT_EINVAL, "ray split must be 0, 1, 2, 4 or 8");
        g_opt_split = value;
        return RT_OK;
    case RT_OPT_FWD_GROUP:
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return fail(RT_EINVAL, "forward lanes per pixel must be 0, 1, 2 or 4");
        g_opt_group = value;
        return RT_OK;
    default:
        return fail(RT_EINVAL, "unknown option %d", key);
    }
}

int64_t rt_get_option(int32_t key) {
    switch (key) {
    case RT_OPT_CHANNEL_BLOCK: return g_opt_cb;
    case RT_OPT_THIN_EXPM1: return g_opt_thin;
    case RT_OPT_CKPT_SEGMENT: return g_opt_ckpt;
    case RT_OPT_RAY_SPLIT: return g_opt_split;
    case RT_OPT_GRAD_ACCUM: return g_opt_accum;
    case RT_OPT_ADJ_SCRATCH_CAP: return g_opt_adj_cap;
    case RT_OPT_ADJ_CHANNEL_BLOCK: return g_opt_adj_cb;
    case RT_OPT_ADJ_PIXEL_LANES: return g_opt_adj_lanes;
    case RT_OPT_FWD_GROUP: return g_opt_group;
    default: return -1;
    }
}

rt_status rt_render_cube(const rt_problem *p, float *cube, void *stream) {
    rt_status st = validate(p);
    if (st != RT_OK) return st;
    if (!cube) return fail(RT_EINVAL, "cube is NULL");
    if (p->mlp) return render_cube_mlp(p, cube, (hipStream_t)stream);
    Geometry g;
    Shade s;
    st = build_launch(p, &g, &s);
    if (st != RT_OK) return st;
    return march_cube(p, g, s, cube, (hipStream_t)stream);
}

} // extern "C"
