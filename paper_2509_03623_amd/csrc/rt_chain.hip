// rt_chain.hip -- fields derived from a temperature grid, and their adjoint.
//
// Methods, "Parametric Disk Modeling" (Eqs. gas_density_temp, column_density,
// co_layer, gas_velocity_pressure) as used by "Neural Temperature Recovery"
// (physics-informed constraints): n_H2 from vertical hydrostatic equilibrium
// normalised to the surface density, the CO surfaces from the vertical column
// and the freeze-out temperature, v_phi from gravity and the radial pressure
// gradient.  The discretisation is stated in include/rtcube.h.
//
// The work is a few operations per grid node (3.3e4 nodes at 256 x 128): the
// scans along a column run in one 64-lane wave that stages the column's rows
// in LDS (one workgroup per radial node), the stencils in one lane per node;
// a call is a few launches of tens of microseconds next to a render of
// milliseconds.  Lengths are in au inside the kernels (cm^3-scale powers
// would overflow float), with the unit factors folded into the constants on
// the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/rtcube.h"
#include "rt_host.h"
#include "rt_kernels.h"

namespace rt {

namespace {

// cgs constants (CODATA 2018, IAU 2015 nominal)
constexpr double kG = 6.67430e-8, kMsun = 1.98847e33, kAu = 1.495978707e13, kKb = 1.380649e-16,
                 kMh = 1.6735575e-24;
constexpr double kPhotoFactor = 0.706;   // vertical H2 column -> total gas column

// largest column staged in LDS (5 rows of floats: 40 KiB)
constexpr int kChainMaxNz = 2048;

struct ChainArgs {
    int nr, nz;
    float r_min, dlog2r;      // r_i = r_min 2^(i dlog2r)
    float du;                 // ln r step
    float dzeta, zr_max;      // z/r step and top
    float cg;                 // G M m_mol / (k_B au): gravity integrand in K au^-1 with lengths in au
    float cn;                 // -ln(au) - ln(m_mol): ln n = ln Sigma - ln(2 int e^l dz[au]) + l + cn
    float ln_sig0, gamma, inv_rc;   // ln Sigma = ln_sig0 - gamma ln x - x^(2 - gamma), x = r / r_c
    float au_cm;              // column increments: n [cm^-3] dz [au] au_cm
    float thr;                // N_dissoc / 0.706
    float t_freeze;
    float cv;                 // G M / au in (km/s)^2 au: v_K^2 = cv r^2 / (r^2 + z^2)^(3/2)
    float ct;                 // k_B / m_mol in (km/s)^2 / K
};

__device__ __forceinline__ float node_r(const ChainArgs &a, int i) { return a.r_min * exp2f((float)i * a.dlog2r); }

// the gravity integrand g z / T of node height z (au) for column radius r
__device__ __forceinline__ float grav_h(const ChainArgs &a, float r, float z, float T) {
    const float q = r * r + z * z;
    return a.cg * z / (T * q * sqrtf(q));
}

__device__ __forceinline__ float ln_sigma(const ChainArgs &a, float r) {
    const float lx = logf(r * a.inv_rc);
    return a.ln_sig0 - a.gamma * lx - expf((2.0f - a.gamma) * lx);
}

// Wave-wide inclusive prefix sum of one value per lane.
__device__ __forceinline__ float wave_incl_scan(float v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Sums over the lanes below (up) or above (down) this one, formed from the
// shifted values so that no difference of two large partial sums is taken:
// the downward column of the inner segments is ~1e4 times the column above
// the photodissociation surface, and total - prefix lost it to rounding.
__device__ __forceinline__ float wave_excl_scan_up(float v) {
    const int lane = threadIdx.x & 63;
    float x = __shfl_up(v, 1, 64);
    return wave_incl_scan(lane == 0 ? 0.0f : x);
}

__device__ __forceinline__ float wave_excl_scan_down(float v) {
    const int lane = threadIdx.x & 63;
    float x = __shfl_down(v, 1, 64);
    x = lane == 63 ? 0.0f : x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float u = __shfl_down(x, d, 64);
        if (lane + d < 64) x += u;
    }
    return x;
}

// The column pass of radial node i by one 64-lane wave.  The column's rows
// live in LDS and each lane owns a contiguous segment of nodes.  The two
// trapezoid integrals (the hydrostatic one up the column, the downward H2
// column) are prefix and suffix sums (segment sums, a wave scan of the segment
// totals, then the segment again), the normalisation of the density is a wave
// sum, and both crossings are counts: the downward column only grows towards
// the midplane, so the nodes above the photodissociation threshold are the
// first up_a + 1, and the first warm node is a minimum over the lanes.  The
// same quantities as a serial scan of the column, up to the order of the
// roundings.  Leaves T, h, l = ln rho - ln rho_0, n and the downward column N
// in the five LDS rows (synchronised) and writes ln n when ln_n is given.
struct ColumnWave {
    int up_a;    // node below the photodissociation crossing (-1: midplane unshielded)
    int lo_b;    // first warm node (-1: warm midplane, nz: never warm)
    float r, dz;
};

__device__ ColumnWave column_wave(const ChainArgs &a, const float *__restrict__ T, int i, float *sm,
                                  float *__restrict__ ln_n) {
    const int nz = a.nz, lane = threadIdx.x;
    float *sT = sm, *sH = sm + nz, *sL = sm + 2 * nz, *sE = sm + 3 * nz, *sN = sm + 4 * nz;
    const size_t o = (size_t)i * nz;
    const int per = (nz + 63) / 64, j0 = min(nz, lane * per), j1 = min(nz, j0 + per);
    const float r = node_r(a, i), dz = a.dzeta * r;
    for (int j = j0; j < j1; ++j) {
        const float t = T[o + j];
        sT[j] = t;
        sH[j] = grav_h(a, r, (float)j * dz, t);
    }
    __syncthreads();
    // hydrostatic integral I_j = sum_{k=1..j} (h_{k-1} + h_k) dz / 2, l_j = -I_j - ln T_j + ln T_0
    float seg = 0.0f;
    for (int j = max(j0, 1); j < j1; ++j) seg += 0.5f * (sH[j - 1] + sH[j]) * dz;
    float I = wave_excl_scan_up(seg);
    const float lnT0 = logf(sT[0]);
    for (int j = j0; j < j1; ++j) {
        if (j > 0) I += 0.5f * (sH[j - 1] + sH[j]) * dz;
        const float l = -I - logf(sT[j]) + lnT0;
        sL[j] = l;
        sE[j] = expf(l);
    }
    __syncthreads();
    // normalisation: ln rho_0 + cn = ln Sigma - ln(2 int e^l dz) + cn
    float tr = 0.0f;
    for (int j = max(j0, 1); j < j1; ++j) tr += 0.5f * (sE[j - 1] + sE[j]) * dz;
    tr = __shfl(wave_incl_scan(tr), 63, 64);
    const float L0 = ln_sigma(a, r) - logf(2.0f * tr) + a.cn;
    __syncthreads();
    for (int j = j0; j < j1; ++j) {
        const float ln = sL[j] + L0;
        if (ln_n) ln_n[o + j] = ln;
        sE[j] = expf(ln);
    }
    __syncthreads();
    // downward column N_j = sum_{k=j..nz-2} (n_k + n_{k+1}) dz au / 2 (N_{nz-1} = 0)
    const int je = min(j1, nz - 1);
    float cs = 0.0f;
    for (int j = j0; j < je; ++j) cs += 0.5f * (sE[j] + sE[j + 1]) * dz * a.au_cm;
    float N = wave_excl_scan_down(cs);       // the column of the segments above this one (higher j)
    int above = 0;
    for (int j = je - 1; j >= j0; --j) {
        N += 0.5f * (sE[j] + sE[j + 1]) * dz * a.au_cm;
        sN[j] = N;
        above += N > a.thr ? 1 : 0;
    }
    if (lane == 0) sN[nz - 1] = 0.0f;
    // first warm node above the midplane
    int warm = nz;
    for (int j = max(j0, 1); j < j1; ++j)
        if (sT[j] > a.t_freeze) { warm = j; break; }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        above += __shfl_xor(above, d, 64);
        warm = min(warm, __shfl_xor(warm, d, 64));
    }
    __syncthreads();
    return ColumnWave{above - 1, sT[0] > a.t_freeze ? -1 : warm, r, dz};
}

// one 64-lane workgroup per radial node
__global__ __launch_bounds__(64) void chain_columns(ChainArgs a, const float *__restrict__ T, float *__restrict__ ln_n,
                                                    float *__restrict__ zlo, float *__restrict__ zup) {
    extern __shared__ float sm[];
    const int i = blockIdx.x, nz = a.nz;
    const float *sT = sm, *sN = sm + 4 * nz;
    const ColumnWave c = column_wave(a, T, i, sm, ln_n);
    if (threadIdx.x != 0) return;
    const float r = c.r, dz = c.dz;
    if (c.up_a < 0) {
        zup[i] = -a.zr_max * r;
    } else {
        const float Na = sN[c.up_a], Nb = sN[c.up_a + 1];
        float f;
        if (Nb > 0.0f) {
            // ln(thr / N) of the two nodes: the logs of ratios near 1 are exact
            // to rounding, where ln thr - ln N loses the digits of ln thr ~ 48
            const float w = logf(a.thr / Na), u = logf(a.thr / Nb);
            f = w / (w - u);
        } else {
            f = (a.thr - Na) / (Nb - Na);
        }
        zup[i] = ((float)c.up_a + f) * dz;
    }
    if (c.lo_b < 0) {
        zlo[i] = -a.zr_max * r;
    } else if (c.lo_b == nz) {
        zlo[i] = 2.0f * a.zr_max * r;
    } else {
        const int w = c.lo_b;
        zlo[i] = ((float)(w - 1) + (a.t_freeze - sT[w - 1]) / (sT[w] - sT[w - 1])) * dz;
    }
}

__device__ __forceinline__ float lnP(const float *ln_n, const float *T, int nz, int i, int j) {
    return ln_n[(size_t)i * nz + j] + logf(T[(size_t)i * nz + j]);
}

// d ln P / d u and d ln P / d zeta at node (i, j): central differences, one-sided at the edges
__device__ __forceinline__ void dlnP(const ChainArgs &a, const float *ln_n, const float *T, int i, int j, float *du,
                                     float *dzeta) {
    const int il = max(i - 1, 0), ih = min(i + 1, a.nr - 1);
    const int jl = max(j - 1, 0), jh = min(j + 1, a.nz - 1);
    *du = (lnP(ln_n, T, a.nz, ih, j) - lnP(ln_n, T, a.nz, il, j)) / ((float)(ih - il) * a.du);
    *dzeta = (lnP(ln_n, T, a.nz, i, jh) - lnP(ln_n, T, a.nz, i, jl)) / ((float)(jh - jl) * a.dzeta);
}

__device__ __forceinline__ float vphi2(const ChainArgs &a, float r, float zeta, float T, float du, float dzeta) {
    const float z = zeta * r;
    const float q = r * r + z * z;
    return a.cv * r * r / (q * sqrtf(q)) + a.ct * T * (du - zeta * dzeta);
}

__global__ __launch_bounds__(256) void chain_vphi(ChainArgs a, const float *__restrict__ T,
                                                  const float *__restrict__ ln_n, float *__restrict__ vphi) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.nr * a.nz) return;
    const int i = idx / a.nz, j = idx - i * a.nz;
    float du, dz;
    dlnP(a, ln_n, T, i, j, &du, &dz);
    const float v2 = vphi2(a, node_r(a, i), (float)j * a.dzeta, T[idx], du, dz);
    vphi[idx] = v2 > 0.0f ? sqrtf(v2) : 0.0f;
}

// ---- adjoint

// per node: cotangents of the two difference quotients (eu, ez) and the
// direct temperature term of v^2 (gT)
__global__ __launch_bounds__(256) void chain_vphi_adj(ChainArgs a, const float *__restrict__ T,
                                                      const float *__restrict__ ln_n, const float *__restrict__ vbar,
                                                      float *__restrict__ eu, float *__restrict__ ez,
                                                      float *__restrict__ gT) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.nr * a.nz) return;
    const int i = idx / a.nz, j = idx - i * a.nz;
    float du, dz;
    dlnP(a, ln_n, T, i, j, &du, &dz);
    const float zeta = (float)j * a.dzeta;
    const float v2 = vphi2(a, node_r(a, i), zeta, T[idx], du, dz);
    const float vb2 = (vbar && v2 > 0.0f) ? vbar[idx] * 0.5f / sqrtf(v2) : 0.0f;
    gT[idx] = vb2 * a.ct * (du - zeta * dz);
    eu[idx] = vb2 * a.ct * T[idx];
    ez[idx] = -vb2 * a.ct * T[idx] * zeta;
}

// per node: gather the difference-quotient cotangents into d/d ln P, then
// split it into d/d ln n (gn) and d/dT (added to gT)
__global__ __launch_bounds__(256) void chain_lnp_adj(ChainArgs a, const float *__restrict__ T,
                                                     const float *__restrict__ eu, const float *__restrict__ ez,
                                                     float *__restrict__ gn, float *__restrict__ gT) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.nr * a.nz) return;
    const int i = idx / a.nz, j = idx - i * a.nz;
    float g = 0.0f;
    for (int ii = max(i - 1, 0); ii <= min(i + 1, a.nr - 1); ++ii) {
        const int il = max(ii - 1, 0), ih = min(ii + 1, a.nr - 1);
        const float w = ((ih == i) ? 1.0f : 0.0f) - ((il == i) ? 1.0f : 0.0f);
        if (w != 0.0f) g += w * eu[(size_t)ii * a.nz + j] / ((float)(ih - il) * a.du);
    }
    for (int jj = max(j - 1, 0); jj <= min(j + 1, a.nz - 1); ++jj) {
        const int jl = max(jj - 1, 0), jh = min(jj + 1, a.nz - 1);
        const float w = ((jh == j) ? 1.0f : 0.0f) - ((jl == j) ? 1.0f : 0.0f);
        if (w != 0.0f) g += w * ez[(size_t)i * a.nz + jj] / ((float)(jh - jl) * a.dzeta);
    }
    gn[idx] = g;
    gT[idx] += g / T[idx];
}

// per column: reverse of the column pass (crossings held fixed), one 64-lane
// workgroup per radial node.  The forward quantities come from the same wave
// pass as the forward kernel; the reverse is elementwise except for two wave
// sums (the normalisation) and one suffix sum (the cotangent of the
// hydrostatic integral), taken as segment sums and a wave scan of the segments
// above, so no difference of large partial sums is formed.
__global__ __launch_bounds__(64) void chain_columns_adj(ChainArgs a, const float *__restrict__ T,
                                                        const float *__restrict__ nbar, const float *__restrict__ zlobar,
                                                        const float *__restrict__ zupbar,
                                                        const float *__restrict__ gn, const float *__restrict__ gT,
                                                        float *__restrict__ dT, int accumulate) {
    extern __shared__ float sm[];
    const int i = blockIdx.x, nz = a.nz, lane = threadIdx.x;
    const size_t o = (size_t)i * nz;
    float *sT = sm, *sH = sm + nz, *sL = sm + 2 * nz, *sE = sm + 3 * nz;
    const float *sN = sm + 4 * nz;
    const ColumnWave c = column_wave(a, T, i, sm, nullptr);
    const int per = (nz + 63) / 64, j0 = min(nz, lane * per), j1 = min(nz, j0 + per);
    const float dz = c.dz;
    // photodissociation surface -> the two columns it interpolates
    const int ka = c.up_a, kb = c.up_a + 1;
    float Nab = 0.0f, Nbb = 0.0f;
    const float zub = zupbar ? zupbar[i] : 0.0f;
    if (ka >= 0 && zub != 0.0f) {
        const float Na = sN[ka], Nb = sN[kb];
        if (Nb > 0.0f) {
            // f = w / (w - u), w = ln(thr / Na) <= 0 <= u = ln(thr / Nb), as in the forward
            const float w = logf(a.thr / Na), u = logf(a.thr / Nb), d = w - u;
            Nab = zub * dz * (u / (d * d)) / Na;
            Nbb = zub * dz * (-w / (d * d)) / Nb;
        } else {
            const float d = Nb - Na;
            Nab = zub * dz * ((a.thr - Nb) / (d * d));
            Nbb = zub * dz * (-(a.thr - Na) / (d * d));
        }
    }
    // d L / d ln n_j: given plus from v_phi, and from the two columns (N_k
    // sums the trapezoid segments from node k up: n_j enters the segments
    // below and above it); kept in sE in place of n_j
    float gsum = 0.0f, trap = 0.0f;
    for (int j = j0; j < j1; ++j) {
        float g = (nbar ? nbar[o + j] : 0.0f) + gn[o + j];
        if (ka >= 0) {
            const float dka = (float)((j >= ka + 1) ? 1 : 0) + (float)((j >= ka && j <= nz - 2) ? 1 : 0);
            const float dkb = (float)((j >= kb + 1) ? 1 : 0) + (float)((j >= kb && j <= nz - 2) ? 1 : 0);
            g += sE[j] * 0.5f * dz * a.au_cm * (Nab * dka + Nbb * dkb);
        }
        gsum += g;
        trap += ((j == 0 || j == nz - 1) ? 0.5f : 1.0f) * expf(sL[j]);
        sE[j] = g;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        gsum += __shfl_xor(gsum, d, 64);
        trap += __shfl_xor(trap, d, 64);
    }
    // ln n_j = l_j + ln rho_0 + const, ln rho_0 = ln Sigma - ln(2 dz sum w_j e^l_j):
    // cotangent of l_j into sL
    float seg = 0.0f;
    for (int j = j0; j < j1; ++j) {
        const float w = (j == 0 || j == nz - 1) ? 0.5f : 1.0f;
        const float lb = sE[j] - gsum * w * expf(sL[j]) / trap;
        sL[j] = lb;
        seg += lb;
    }
    // l_j = -I_j - ln T_j + ln T_0, I_j = sum over the segments below j of
    // (h_s + h_s+1) dz / 2: node k's h enters I_j for j >= k (twice for j > k)
    float R = wave_excl_scan_down(seg);   // suffix sum of the cotangent of l from j1 up
    const float t_f = a.t_freeze;
    const float zlb = zlobar ? zlobar[i] : 0.0f;
    for (int k = j1 - 1; k >= j0; --k) {
        const float Rnext = R;
        R += sL[k];
        const float hb = -0.5f * dz * ((k <= nz - 2 ? Rnext : 0.0f) + (k >= 1 ? R : 0.0f));
        const float Tk = sT[k];
        float g = -sL[k] / Tk - hb * sH[k] / Tk + gT[o + k];
        // freeze-out surface: linear in T between nodes lo_b - 1 and lo_b
        if (zlb != 0.0f && c.lo_b > 0 && c.lo_b < nz) {
            const int b = c.lo_b, aa = b - 1;
            const float d = sT[b] - sT[aa];
            if (k == aa) g += zlb * dz * (t_f - sT[b]) / (d * d);
            if (k == b) g -= zlb * dz * (t_f - sT[aa]) / (d * d);
        }
        if (k == 0) g += R / sT[0];     // ln T_0 enters every l_j
        dT[o + k] = accumulate ? dT[o + k] + g : g;
    }
}

// two-layer parametric temperature at every node (one lane per node)
__global__ __launch_bounds__(256) void parametric_t(int nr, int nz, float r_min, float dlog2r, float dzeta,
                                                    rt_param_temp pt, float *__restrict__ T) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nr * nz) return;
    const int i = idx / nz, j = idx - i * nz;
    const float r = r_min * exp2f((float)i * dlog2r);
    const float z = (float)j * dzeta * r;
    const float lx = logf(r / (float)pt.r_scale_au);
    const float px = expf((float)pt.q * lx);
    const float tmid = (float)pt.t_mid0_k * px, tatm = (float)pt.t_atm0_k * px;
    const float zq = (float)pt.zq0_au * expf(1.3f * lx);
    float blend = 0.0f;
    if (z < zq) {
        const float c = cospif(0.5f * z / zq);
        blend = c > 0.0f ? expf(2.0f * (float)pt.delta * logf(c)) : 0.0f;
    }
    T[idx] = tatm + (tmid - tatm) * blend;
}

ChainArgs chain_args(const rt_derive *d) {
    const rt_grid &g = d->grid;
    ChainArgs a;
    a.nr = g.nr;
    a.nz = g.nz;
    a.r_min = (float)g.r_min_au;
    a.dlog2r = (float)(std::log2(g.r_max_au / g.r_min_au) / (g.nr - 1));
    a.du = (float)(std::log(g.r_max_au / g.r_min_au) / (g.nr - 1));
    a.dzeta = (float)(g.zr_max / (g.nz - 1));
    a.zr_max = (float)g.zr_max;
    const double m_mol = d->mu * kMh;
    a.cg = (float)(kG * d->mstar_msun * kMsun * m_mol / (kKb * kAu));
    a.cn = (float)(-std::log(kAu) - std::log(m_mol));
    const double rc = d->rc_au * kAu;
    a.ln_sig0 = (float)std::log(d->mgas_msun * kMsun * (2.0 - d->gamma) / (2.0 * M_PI * rc * rc));
    a.gamma = (float)d->gamma;
    a.inv_rc = (float)(1.0 / d->rc_au);
    a.au_cm = (float)kAu;
    a.thr = (float)(d->n_dissoc_cm2 / kPhotoFactor);
    a.t_freeze = (float)d->t_freeze_k;
    a.cv = (float)(kG * d->mstar_msun * kMsun / kAu / 1e10);
    a.ct = (float)(kKb / m_mol / 1e10);
    return a;
}

rt_status validate_derive(const rt_derive *d) {
    if (!d) return fail(RT_EINVAL, "derive parameters are NULL");
    const rt_grid &g = d->grid;
    if (g.nr < 2 || g.nz < 2) return fail(RT_EINVAL, "grid needs nr, nz >= 2");
    if (!(g.r_min_au > 0.0) || !(g.r_max_au > g.r_min_au) || !(g.zr_max > 0.0))
        return fail(RT_EINVAL, "grid needs 0 < r_min < r_max and zr_max > 0");
    if ((size_t)g.nr * g.nz > (size_t)1 << 28) return fail(RT_EINVAL, "grid too large");
    if (g.nz > kChainMaxNz) return fail(RT_EINVAL, "derived fields take at most %d z/r nodes", kChainMaxNz);
    if (!d->temp_k) return fail(RT_EINVAL, "temp_k is NULL");
    if (!(d->mstar_msun >= 0.0) || !(d->mgas_msun > 0.0) || !(d->rc_au > 0.0) || !(d->gamma < 2.0) || !(d->mu > 0.0))
        return fail(RT_EINVAL, "need mstar >= 0, mgas > 0, rc > 0, gamma < 2, mu > 0");
    if (!(d->t_freeze_k > 0.0) || !(d->n_dissoc_cm2 > 0.0)) return fail(RT_EINVAL, "thresholds must be > 0");
    return RT_OK;
}

} // namespace

} // namespace rt

using namespace rt;

extern "C" rt_status rt_derive_fields(const rt_derive *d, const rt_derived *out, void *stream) {
    rt_status st = validate_derive(d);
    if (st != RT_OK) return st;
    if (!out || !out->ln_nh2 || !out->vphi_kms || !out->z_lo_au || !out->z_up_au)
        return fail(RT_EINVAL, "every derived output must be given");
    const ChainArgs a = chain_args(d);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(chain_columns, dim3(a.nr), dim3(64), 5 * sizeof(float) * a.nz, s, a, d->temp_k, out->ln_nh2,
                       out->z_lo_au, out->z_up_au);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "derive columns");
    const int n = a.nr * a.nz;
    hipLaunchKernelGGL(chain_vphi, dim3((n + 255) / 256), dim3(256), 0, s, a, d->temp_k, out->ln_nh2, out->vphi_kms);
    e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "derive v_phi");
}

static rt_status derive_adjoint(const rt_derive *d, const rt_derived *cot, float *d_temp_k, int accumulate,
                                void *stream) {
    rt_status st = validate_derive(d);
    if (st != RT_OK) return st;
    if (!cot) return fail(RT_EINVAL, "cotangents are NULL");
    if (!d_temp_k) return fail(RT_EINVAL, "d_temp_k is NULL");
    const ChainArgs a = chain_args(d);
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)a.nr * a.nz;
    hipError_t e;
    // scratch: eu, ez, gn, gT, and the forward ln n for the stencils
    float *w = (float *)stream_workspace(s, kWsChain, sizeof(float) * 5 * n, &e);
    if (!w) return fail_hip(e, "derive scratch");
    float *eu = w, *ez = w + n, *gn = w + 2 * n, *gT = w + 3 * n, *lnn = w + 4 * n;
    // forward ln n (and surfaces into discarded slots of gn) for the v_phi stencils
    hipLaunchKernelGGL(chain_columns, dim3(a.nr), dim3(64), 5 * sizeof(float) * a.nz, s, a, d->temp_k, lnn, gn,
                       gn + a.nr);
    hipLaunchKernelGGL(chain_vphi_adj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, d->temp_k, lnn,
                       cot->vphi_kms, eu, ez, gT);
    hipLaunchKernelGGL(chain_lnp_adj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, d->temp_k, eu, ez, gn, gT);
    hipLaunchKernelGGL(chain_columns_adj, dim3(a.nr), dim3(64), 5 * sizeof(float) * a.nz, s, a, d->temp_k,
                       cot->ln_nh2, cot->z_lo_au, cot->z_up_au, gn, gT, d_temp_k, accumulate);
    e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "derive adjoint");
}

extern "C" rt_status rt_derive_fields_adjoint(const rt_derive *d, const rt_derived *cot, float *d_temp_k,
                                              void *stream) {
    return derive_adjoint(d, cot, d_temp_k, 0, stream);
}

extern "C" rt_status rt_derive_fields_adjoint_add(const rt_derive *d, const rt_derived *cot, float *d_temp_k,
                                                  void *stream) {
    return derive_adjoint(d, cot, d_temp_k, 1, stream);
}

extern "C" rt_status rt_parametric_temperature(const rt_grid *grid, const rt_param_temp *pt, float *temp_k,
                                               void *stream) {
    if (!grid || !pt || !temp_k) return fail(RT_EINVAL, "grid, parameters and temp_k must not be NULL");
    if (grid->nr < 2 || grid->nz < 2 || !(grid->r_min_au > 0.0) || !(grid->r_max_au > grid->r_min_au) ||
        !(grid->zr_max > 0.0))
        return fail(RT_EINVAL, "grid needs nr, nz >= 2, 0 < r_min < r_max, zr_max > 0");
    if (!(pt->t_mid0_k > 0.0) || !(pt->t_atm0_k > 0.0) || !(pt->r_scale_au > 0.0) || !(pt->zq0_au > 0.0) ||
        !(pt->delta > 0.0))
        return fail(RT_EINVAL, "temperatures, r_scale, zq0 and delta must be > 0");
    const int n = grid->nr * grid->nz;
    hipLaunchKernelGGL(parametric_t, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, grid->nr, grid->nz,
                       (float)grid->r_min_au, (float)(std::log2(grid->r_max_au / grid->r_min_au) / (grid->nr - 1)),
                       (float)(grid->zr_max / (grid->nz - 1)), *pt, temp_k);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RT_OK : fail_hip(e, "parametric temperature");
}
