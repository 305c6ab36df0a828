/*
 * rt_oracle.c -- plain FP64 CPU oracle of the line radiative-transfer ray
 * march.  TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark call it; the GPU library never does.
 *
 * It computes, in double precision with scalar loops and no blocking, the
 * discretised formal solution of the line transfer equation (Methods, "Line
 * Radiative Transfer": Eq. rt-int with the optical depth of Eq.
 * optical_depth, LTE emissivity j and extinction beta, Gaussian Doppler
 * profile with thermal + turbulent width alpha):
 *
 *   every pixel casts one backward ray (orthographic camera, inclination i);
 *   the ray's chord through the bounding cylinder is cut into nsamp equal
 *   segments; fields are sampled at segment midpoints and held constant over
 *   the segment; a segment with constant j and beta contributes
 *   (j/beta)(1 - exp(-beta ds)) attenuated by exp(-tau) of everything in
 *   front of it, and there is no background term.
 *
 * The readings taken where the paper is silent (grid conventions, border
 * taper, soft CO mask, sign conventions, channel grid) are listed with the
 * rest of the design notes; each step below names the one it uses.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* cgs constants (CODATA 2018, IAU 2015 nominal), typed here on their own */
#define ORC_H    6.62607015e-27
#define ORC_KB   1.380649e-16
#define ORC_C    2.99792458e10
#define ORC_AMU  1.66053906660e-24
#define ORC_AU   1.495978707e13
#define ORC_PI   3.14159265358979323846

typedef struct {
    /* (r, z/r) node grid: r log-spaced on [r_min, r_max], z/r linear on [0, zr_max] */
    int32_t nr, nz;
    double r_min_au, r_max_au, zr_max;
    const float *ln_nh2;   /* [nr][nz] ln n_H2 [cm^-3] */
    const float *temp_k;   /* [nr][nz] T [K] */
    const float *vphi_kms; /* [nr][nz] azimuthal velocity [km/s] */
    const float *z_lo_au;  /* [nr] lower CO surface (freeze-out) [au] */
    const float *z_up_au;  /* [nr] upper CO surface (photodissociation) [au] */
    double x_co, mask_width, v_turb;
    /* line */
    double nu0_hz, a_ul, g_u, g_l, e_u_k, e_l_k, m_co_amu, m_mol_amu;
    int32_t nlev;
    const double *lev_e_k, *lev_g;
    /* camera */
    int32_t nx, ny;
    double fov_au, incl_deg, pa_deg;
    /* spectral */
    int32_t nch;
    const double *v_kms;
    double v_sys_kms;
    int32_t nsamp;
    double intensity_scale;
    /* optional neural CO layer (flat float32 weights, see orc_mlp) */
    const float *mlp_w;
} orc_problem;

/* ------------------------------------------------------------ small helpers */
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }
static double silu(double x) { return x * sigm(x); }

/* Level population normaliser Z(T) = sum_J g_J exp(-E_J / kT): Boltzmann
 * statistics over the tabulated levels (Methods, Line RT). */
double orc_partition(const orc_problem *P, double t)
{
    double z = 0.0;
    for (int j = 0; j < P->nlev; ++j) z += P->lev_g[j] * exp(-P->lev_e_k[j] / t);
    return z;
}

/* Neural CO-layer network: 16 Fourier frequencies f_k = 2^(3k/15) applied as
 * sin(pi f c), cos(pi f c) to each of the two normalised grid coordinates,
 * 4 hidden SiLU layers of width 128, 3 linear outputs.  Weights are float32,
 * W_l [out][in] row-major followed by b_l [out], layer after layer. */
#define ORC_NF 16
#define ORC_W 128
void orc_mlp(const float *w, double rh, double zh, double out[3])
{
    double x[4 * ORC_NF], h[ORC_W], g[ORC_W];
    for (int k = 0; k < ORC_NF; ++k) {
        double f = pow(2.0, 3.0 * k / 15.0);
        x[k] = sin(ORC_PI * f * rh);
        x[ORC_NF + k] = cos(ORC_PI * f * rh);
        x[2 * ORC_NF + k] = sin(ORC_PI * f * zh);
        x[3 * ORC_NF + k] = cos(ORC_PI * f * zh);
    }
    const float *p = w;
    /* layer 1: 64 -> 128 */
    for (int o = 0; o < ORC_W; ++o) {
        double s = 0.0;
        for (int i = 0; i < 4 * ORC_NF; ++i) s += (double)p[o * 4 * ORC_NF + i] * x[i];
        h[o] = s;
    }
    p += ORC_W * 4 * ORC_NF;
    for (int o = 0; o < ORC_W; ++o) h[o] = silu(h[o] + (double)p[o]);
    p += ORC_W;
    /* layers 2..4: 128 -> 128 */
    for (int l = 0; l < 3; ++l) {
        for (int o = 0; o < ORC_W; ++o) {
            double s = 0.0;
            for (int i = 0; i < ORC_W; ++i) s += (double)p[o * ORC_W + i] * h[i];
            g[o] = s;
        }
        p += ORC_W * ORC_W;
        for (int o = 0; o < ORC_W; ++o) h[o] = silu(g[o] + (double)p[o]);
        p += ORC_W;
    }
    /* output: 128 -> 3 */
    for (int o = 0; o < 3; ++o) {
        double s = 0.0;
        for (int i = 0; i < ORC_W; ++i) s += (double)p[o * ORC_W + i] * h[i];
        out[o] = s + (double)p[3 * ORC_W + o];
    }
}

/* ------------------------------------------------------------ one sample */
typedef struct {
    double S;       /* source function j/beta [erg s^-1 cm^-2 Hz^-1 sr^-1] */
    double kbar;    /* beta without its profile: (h nu0 / 4 pi)(n_l B_lu - n_u B_ul) [cm^-1 Hz] */
    double alpha;   /* Gaussian width [km/s] */
    double vlos;    /* line-of-sight velocity incl. systemic [km/s] */
    double nu;      /* upper-level density [cm^-3] */
} orc_sample;

static void sample_point(const orc_problem *P, double px, double py, double pz, orc_sample *o)
{
    memset(o, 0, sizeof *o);
    const double rho = sqrt(px * px + py * py);
    const double a = fabs(pz);
    if (rho == 0.0) return;                      /* on the axis: empty sample */
    const double dln = log(P->r_max_au / P->r_min_au) / (P->nr - 1);
    const double dzr = P->zr_max / (P->nz - 1);
    /* continuous grid index in (ln r, z/r) */
    const double u = log(rho / P->r_min_au) / dln;
    const double v = (a / rho) / dzr;
    /* clamp-to-edge bilinear weights */
    const double uc = clampd(u, 0.0, P->nr - 1), vc = clampd(v, 0.0, P->nz - 1);
    int i0 = (int)floor(uc); if (i0 > P->nr - 2) i0 = P->nr - 2;
    int j0 = (int)floor(vc); if (j0 > P->nz - 2) j0 = P->nz - 2;
    const double fu = uc - i0, fv = vc - j0;
    const int n00 = i0 * P->nz + j0, n01 = n00 + 1, n10 = n00 + P->nz, n11 = n10 + 1;
    const double w00 = (1 - fu) * (1 - fv), w01 = (1 - fu) * fv, w10 = fu * (1 - fv), w11 = fu * fv;
#define BIL(F) (w00 * (double)(F)[n00] + w01 * (double)(F)[n01] + w10 * (double)(F)[n10] + w11 * (double)(F)[n11])
    const double ln_n = BIL(P->ln_nh2);
    double t = BIL(P->temp_k);
    const double vphi = BIL(P->vphi_kms);
#undef BIL
    double zlo = (1 - fu) * (double)P->z_lo_au[i0] + fu * (double)P->z_lo_au[i0 + 1];
    double zup = (1 - fu) * (double)P->z_up_au[i0] + fu * (double)P->z_up_au[i0 + 1];
    if (P->mlp_w) {
        /* neural CO layer: network on the clamped, normalised grid coordinates */
        double out[3];
        const double rh = clampd(u, -1.0, P->nr) / (P->nr - 1);
        const double zh = clampd(v, 0.0, P->nz) / (P->nz - 1);
        orc_mlp(P->mlp_w, rh, zh, out);
        zup = P->zr_max * rho * sigm(out[0]);
        zlo = P->zr_max * rho * sigm(out[1]);
        t = t * exp(0.5 * tanh(out[2]));
    }
    /* density fades linearly to zero one cell beyond the grid */
    const double taper = clampd(u + 1.0, 0.0, 1.0) * clampd(P->nr - u, 0.0, 1.0) * clampd(P->nz - v, 0.0, 1.0);
    const double nh2 = exp(ln_n) * taper;
    /* CO between the freeze-out and photodissociation surfaces (Eq. co_layer),
     * as a logistic mask of width mask_width * rho * dzr */
    const double w = P->mask_width * rho * dzr;
    const double mask = sigm((zup - a) / w) * sigm((a - zlo) / w);
    const double nco = P->x_co * mask * nh2;
    /* LTE level populations */
    const double zpart = orc_partition(P, t);
    const double nu = nco * P->g_u * exp(-P->e_u_k / t) / zpart;
    const double nl = nco * P->g_l * exp(-P->e_l_k / t) / zpart;
    /* Einstein coefficients */
    const double nu0 = P->nu0_hz;
    const double bul = P->a_ul * ORC_C * ORC_C / (2.0 * ORC_H * nu0 * nu0 * nu0);
    const double blu = P->g_u / P->g_l * bul;
    const double pre = ORC_H * nu0 / (4.0 * ORC_PI);
    const double jbar = pre * nu * P->a_ul;            /* j without its profile */
    const double kbar = pre * (nl * blu - nu * bul);   /* beta without its profile */
    o->kbar = kbar;
    o->S = kbar > 0.0 ? jbar / kbar : 0.0;
    o->nu = nu;
    /* line width: thermal + turbulent (Mach number v_turb of c_s^2 = 2kT/m_mol) */
    const double th = 2.0 * ORC_KB * t / (P->m_co_amu * ORC_AMU);
    const double cs2 = 2.0 * ORC_KB * t / (P->m_mol_amu * ORC_AMU);
    o->alpha = sqrt(th + P->v_turb * P->v_turb * cs2) / 1e5;
    /* projected velocity: counter-clockwise rotation about +z, omega_x = 0 */
    const double si = sin(P->incl_deg * ORC_PI / 180.0);
    o->vlos = P->v_sys_kms + vphi * si * px / rho;
}

/* Gaussian line profile at channel velocity vc [Hz^-1]: the paper's phi(nu)
 * written in velocity with nu_c = nu0 (1 - v_c/c). */
static double profile(const orc_problem *P, const orc_sample *s, double vc)
{
    if (s->alpha <= 0.0) return 0.0;
    const double d = (s->vlos - vc) / s->alpha;
    return (ORC_C / P->nu0_hz) / (s->alpha * 1e5 * sqrt(ORC_PI)) * exp(-d * d);
}

/* ------------------------------------------------------------ one ray */
typedef struct { double x, y; } orc_xy;

static orc_xy pixel_xy(const orc_problem *P, int p, int q)
{
    const double d = P->fov_au / P->nx;
    const double X = (p + 0.5 - 0.5 * P->nx) * d, Y = (q + 0.5 - 0.5 * P->ny) * d;
    const double pa = P->pa_deg * ORC_PI / 180.0;
    orc_xy r = { cos(pa) * X - sin(pa) * Y, sin(pa) * X + cos(pa) * Y };
    return r;
}

/* Chord of the ray x' e_x + y' e_y + s w through the cylinder rho <= Rc,
 * |z| <= Zc (one cell beyond the grid in r and z/r).  Returns 0 if empty. */
static int chord(const orc_problem *P, double xp, double yp, double *sa, double *sb)
{
    const double dln = log(P->r_max_au / P->r_min_au) / (P->nr - 1);
    const double dzr = P->zr_max / (P->nz - 1);
    const double Rc = P->r_max_au * exp(dln);
    const double Zc = (P->zr_max + dzr) * Rc;
    const double ang = P->incl_deg * ORC_PI / 180.0;
    const double si = sin(ang), ci = cos(ang);
    double lo = -INFINITY, hi = INFINITY;
    if (xp * xp >= Rc * Rc) return 0;
    const double qq = sqrt(Rc * Rc - xp * xp);
    if (si > 0.0) {
        lo = fmax(lo, (-yp * ci - qq) / si);
        hi = fmin(hi, (-yp * ci + qq) / si);
    } else if (fabs(yp * ci) > qq) return 0;
    if (ci > 0.0) {
        lo = fmax(lo, (yp * si - Zc) / ci);
        hi = fmin(hi, (yp * si + Zc) / ci);
    } else if (fabs(yp * si) > Zc) return 0;
    if (!(hi > lo)) return 0;
    *sa = lo; *sb = hi;
    return 1;
}

/* March one ray front to back; I[c] receives the intensity of every channel.
 * If S_out / dtau_out are given they receive the per-sample source function
 * and optical depths [k][c] (for recurrence checks). */
static void march(const orc_problem *P, int p, int q, double *I, double *S_out, double *dtau_out,
                  double *chord_out)
{
    const int nch = P->nch;
    double *tr = (double *)malloc(sizeof(double) * nch);
    for (int c = 0; c < nch; ++c) { I[c] = 0.0; tr[c] = 1.0; }
    orc_xy xy = pixel_xy(P, p, q);
    double sa, sb;
    if (!chord(P, xy.x, xy.y, &sa, &sb)) {
        if (chord_out) { chord_out[0] = chord_out[1] = chord_out[2] = 0.0; }
        if (S_out) for (int k = 0; k < P->nsamp; ++k) S_out[k] = 0.0;
        if (dtau_out) for (int k = 0; k < P->nsamp * nch; ++k) dtau_out[k] = 0.0;
        free(tr);
        return;
    }
    const double ds = (sb - sa) / P->nsamp;
    if (chord_out) { chord_out[0] = sa; chord_out[1] = sb; chord_out[2] = ds; }
    const double ds_cm = ds * ORC_AU;
    const double ang = P->incl_deg * ORC_PI / 180.0;
    const double si = sin(ang), ci = cos(ang);
    for (int k = 0; k < P->nsamp; ++k) {
        const double s = sa + (k + 0.5) * ds;
        const double px = xy.x, py = xy.y * ci + s * si, pz = xy.y * si - s * ci;
        orc_sample smp;
        sample_point(P, px, py, pz, &smp);
        if (S_out) S_out[k] = smp.S;
        for (int c = 0; c < nch; ++c) {
            const double dtau = smp.kbar * profile(P, &smp, P->v_kms[c]) * ds_cm;
            if (dtau_out) dtau_out[(size_t)k * nch + c] = dtau;
            /* exact segment solution for constant j and beta */
            I[c] += tr[c] * smp.S * (-expm1(-dtau));
            tr[c] *= exp(-dtau);
        }
    }
    for (int c = 0; c < nch; ++c) I[c] *= P->intensity_scale;
    free(tr);
}

/* ------------------------------------------------------------ exported API */
int orc_render(const orc_problem *P, double *cube, int nthreads)
{
    if (!P || !cube || P->nr < 2 || P->nz < 2 || P->nx < 1 || P->ny < 1 || P->nch < 1 || P->nsamp < 1)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int q = 0; q < P->ny; ++q) {
        double *I = (double *)malloc(sizeof(double) * P->nch);
        for (int p = 0; p < P->nx; ++p) {
            march(P, p, q, I, NULL, NULL, NULL);
            for (int c = 0; c < P->nch; ++c) cube[((size_t)c * P->ny + q) * P->nx + p] = I[c];
        }
        free(I);
    }
    (void)nthreads;
    return 0;
}

/* Intensities of an explicit pixel list: out[n][c]. */
int orc_render_pixels(const orc_problem *P, int npix, const int32_t *px, const int32_t *py, double *out,
                      int nthreads)
{
    if (!P || !out || npix < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int n = 0; n < npix; ++n) march(P, px[n], py[n], out + (size_t)n * P->nch, NULL, NULL, NULL);
    (void)nthreads;
    return 0;
}

/* Per-sample source function S[k] and optical depth dtau[k][c] of one ray,
 * plus (s_a, s_b, ds) of its chord; I[c] is its intensity. */
int orc_ray_dump(const orc_problem *P, int p, int q, double *I, double *S, double *dtau, double *ch)
{
    if (!P) return -1;
    march(P, p, q, I, S, dtau, ch);
    return 0;
}

/* Sample one point: out = {S, kbar, alpha, vlos, n_u}. */
int orc_sample_point(const orc_problem *P, double px, double py, double pz, double *out)
{
    orc_sample s;
    sample_point(P, px, py, pz, &s);
    out[0] = s.S; out[1] = s.kbar; out[2] = s.alpha; out[3] = s.vlos; out[4] = s.nu;
    return 0;
}

/* The constants this file uses, in a fixed order: h, k_B, c, amu, au, pi. */
int orc_constants(double *out, int n)
{
    const double v[6] = { ORC_H, ORC_KB, ORC_C, ORC_AMU, ORC_AU, ORC_PI };
    for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
    return 6;
}

/* ============================================================ 3-D spherical grid
 *
 * Fields on a spherical node grid (r log-spaced on [r_min, r_max], polar angle
 * theta linear on [theta_min, theta_max], azimuth phi_k = 2 pi k / nphi,
 * periodic), layout [nr][ntheta][nphi]: ln n_H2, T, the velocity components
 * (v_r, v_theta, v_phi) and the CO abundance x_CO.  Trilinear interpolation in
 * (ln r, theta, phi), clamped to the edge in r and theta, periodic in phi; the
 * density fades linearly to zero one cell beyond the radial and polar ranges.
 * Every ray's chord through the sphere r <= r_max e^dln is cut into nsamp
 * equal segments; the line physics is that of the 2-D march with
 * n_CO = x_CO n_H2 and v_los = v_sys + v . w (w = (0, sin i, -cos i), the ray
 * direction in the disk frame). */
typedef struct {
    int32_t nr, nt, np;
    double r_min_au, r_max_au, th_min, th_max;
    const float *ln_nh2, *temp_k, *v_r, *v_t, *v_p, *x_co;   /* [nr][nt][np] */
    double v_turb;
    double nu0_hz, a_ul, g_u, g_l, e_u_k, e_l_k, m_co_amu, m_mol_amu;
    int32_t nlev;
    const double *lev_e_k, *lev_g;
    int32_t nx, ny;
    double fov_au, incl_deg, pa_deg;
    int32_t nch;
    const double *v_kms;
    double v_sys_kms;
    int32_t nsamp;
    double intensity_scale;
} orc_problem3;

static void sample_point3(const orc_problem3 *P, double px, double py, double pz, orc_sample *o)
{
    memset(o, 0, sizeof *o);
    const double r = sqrt(px * px + py * py + pz * pz);
    if (r == 0.0) return;
    const double rho = sqrt(px * px + py * py);
    const double th = acos(clampd(pz / r, -1.0, 1.0));
    double ph = atan2(py, px);
    if (ph < 0.0) ph += 2.0 * ORC_PI;
    const double dln = log(P->r_max_au / P->r_min_au) / (P->nr - 1);
    const double dth = (P->th_max - P->th_min) / (P->nt - 1);
    const double dph = 2.0 * ORC_PI / P->np;
    const double u = log(r / P->r_min_au) / dln, w = (th - P->th_min) / dth, s = ph / dph;
    const double uc = clampd(u, 0.0, P->nr - 1), wc = clampd(w, 0.0, P->nt - 1);
    int i0 = (int)floor(uc); if (i0 > P->nr - 2) i0 = P->nr - 2;
    int j0 = (int)floor(wc); if (j0 > P->nt - 2) j0 = P->nt - 2;
    int k0 = (int)floor(s);
    const double fu = uc - i0, fw = wc - j0, fs = s - k0;
    k0 = ((k0 % P->np) + P->np) % P->np;
    const int k1 = (k0 + 1) % P->np;
    double wgt[8];
    size_t idx[8];
    int m = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                wgt[m] = (a ? fu : 1 - fu) * (b ? fw : 1 - fw) * (c ? fs : 1 - fs);
                idx[m] = ((size_t)(i0 + a) * P->nt + (j0 + b)) * P->np + (c ? k1 : k0);
                ++m;
            }
#define TRI(F) (wgt[0] * (double)(F)[idx[0]] + wgt[1] * (double)(F)[idx[1]] + wgt[2] * (double)(F)[idx[2]] + \
                wgt[3] * (double)(F)[idx[3]] + wgt[4] * (double)(F)[idx[4]] + wgt[5] * (double)(F)[idx[5]] + \
                wgt[6] * (double)(F)[idx[6]] + wgt[7] * (double)(F)[idx[7]])
    const double ln_n = TRI(P->ln_nh2), t = TRI(P->temp_k), xco = TRI(P->x_co);
    const double vr = TRI(P->v_r), vt = TRI(P->v_t), vp = TRI(P->v_p);
#undef TRI
    const double taper = clampd(u + 1.0, 0.0, 1.0) * clampd(P->nr - u, 0.0, 1.0) * clampd(w + 1.0, 0.0, 1.0) *
                         clampd(P->nt - w, 0.0, 1.0);
    const double nco = xco * exp(ln_n) * taper;
    double zpart = 0.0;
    for (int j = 0; j < P->nlev; ++j) zpart += P->lev_g[j] * exp(-P->lev_e_k[j] / t);
    const double nu = nco * P->g_u * exp(-P->e_u_k / t) / zpart;
    const double nl = nco * P->g_l * exp(-P->e_l_k / t) / zpart;
    const double nu0 = P->nu0_hz;
    const double bul = P->a_ul * ORC_C * ORC_C / (2.0 * ORC_H * nu0 * nu0 * nu0);
    const double blu = P->g_u / P->g_l * bul;
    const double pre = ORC_H * nu0 / (4.0 * ORC_PI);
    const double jbar = pre * nu * P->a_ul;
    const double kbar = pre * (nl * blu - nu * bul);
    o->kbar = kbar;
    o->S = kbar > 0.0 ? jbar / kbar : 0.0;
    o->nu = nu;
    const double thv = 2.0 * ORC_KB * t / (P->m_co_amu * ORC_AMU);
    const double cs2 = 2.0 * ORC_KB * t / (P->m_mol_amu * ORC_AMU);
    o->alpha = sqrt(thv + P->v_turb * P->v_turb * cs2) / 1e5;
    /* unit vectors at the sample, projected on the ray direction w */
    const double ang = P->incl_deg * ORC_PI / 180.0;
    const double si = sin(ang), ci = cos(ang);
    double vw = vr * (py * si - pz * ci) / r;
    if (rho > 0.0) {
        const double cth = pz / r, sth = rho / r;
        vw += vt * (cth * (py / rho) * si + sth * ci);       /* theta-hat = (cos th cos ph, cos th sin ph, -sin th) */
        vw += vp * (px / rho) * si;                          /* phi-hat = (-sin ph, cos ph, 0) */
    }
    o->vlos = P->v_sys_kms + vw;
}

static void march3(const orc_problem3 *P, int p, int q, double *I, double *S_out, double *dtau_out,
                   double *chord_out)
{
    const int nch = P->nch;
    double *tr = (double *)malloc(sizeof(double) * nch);
    for (int c = 0; c < nch; ++c) { I[c] = 0.0; tr[c] = 1.0; }
    const double d = P->fov_au / P->nx;
    const double X = (p + 0.5 - 0.5 * P->nx) * d, Y = (q + 0.5 - 0.5 * P->ny) * d;
    const double pa = P->pa_deg * ORC_PI / 180.0;
    const double xp = cos(pa) * X - sin(pa) * Y, yp = sin(pa) * X + cos(pa) * Y;
    const double dln = log(P->r_max_au / P->r_min_au) / (P->nr - 1);
    const double Rc = P->r_max_au * exp(dln);
    const double h2 = Rc * Rc - xp * xp - yp * yp;
    if (!(h2 > 0.0)) {
        if (chord_out) { chord_out[0] = chord_out[1] = chord_out[2] = 0.0; }
        if (S_out) for (int k = 0; k < P->nsamp; ++k) S_out[k] = 0.0;
        if (dtau_out) for (int k = 0; k < P->nsamp * nch; ++k) dtau_out[k] = 0.0;
        free(tr);
        return;
    }
    const double sa = -sqrt(h2), sb = sqrt(h2), ds = (sb - sa) / P->nsamp;
    if (chord_out) { chord_out[0] = sa; chord_out[1] = sb; chord_out[2] = ds; }
    const double ds_cm = ds * ORC_AU;
    const double ang = P->incl_deg * ORC_PI / 180.0;
    const double si = sin(ang), ci = cos(ang);
    for (int k = 0; k < P->nsamp; ++k) {
        const double s = sa + (k + 0.5) * ds;
        const double px = xp, py = yp * ci + s * si, pz = yp * si - s * ci;
        orc_sample smp;
        sample_point3(P, px, py, pz, &smp);
        if (S_out) S_out[k] = smp.S;
        for (int c = 0; c < nch; ++c) {
            double dtau = 0.0;
            if (smp.alpha > 0.0) {
                const double dd = (smp.vlos - P->v_kms[c]) / smp.alpha;
                dtau = smp.kbar * (ORC_C / P->nu0_hz) / (smp.alpha * 1e5 * sqrt(ORC_PI)) * exp(-dd * dd) * ds_cm;
            }
            if (dtau_out) dtau_out[(size_t)k * nch + c] = dtau;
            I[c] += tr[c] * smp.S * (-expm1(-dtau));
            tr[c] *= exp(-dtau);
        }
    }
    for (int c = 0; c < nch; ++c) I[c] *= P->intensity_scale;
    free(tr);
}

int orc_render3(const orc_problem3 *P, double *cube, int nthreads)
{
    if (!P || !cube || P->nr < 2 || P->nt < 2 || P->np < 1 || P->nx < 1 || P->ny < 1 || P->nch < 1 || P->nsamp < 1)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int q = 0; q < P->ny; ++q) {
        double *I = (double *)malloc(sizeof(double) * P->nch);
        for (int p = 0; p < P->nx; ++p) {
            march3(P, p, q, I, NULL, NULL, NULL);
            for (int c = 0; c < P->nch; ++c) cube[((size_t)c * P->ny + q) * P->nx + p] = I[c];
        }
        free(I);
    }
    (void)nthreads;
    return 0;
}

int orc_render3_pixels(const orc_problem3 *P, int npix, const int32_t *px, const int32_t *py, double *out,
                       int nthreads)
{
    if (!P || !out || npix < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int n = 0; n < npix; ++n) march3(P, px[n], py[n], out + (size_t)n * P->nch, NULL, NULL, NULL);
    (void)nthreads;
    return 0;
}

int orc_ray_dump3(const orc_problem3 *P, int p, int q, double *I, double *S, double *dtau, double *ch)
{
    if (!P) return -1;
    march3(P, p, q, I, S, dtau, ch);
    return 0;
}

/* One point of a 3-D problem: out = {S, kbar, alpha, vlos, n_u}. */
int orc_sample_point3(const orc_problem3 *P, double px, double py, double pz, double *out)
{
    if (!P || !out) return -1;
    orc_sample s;
    sample_point3(P, px, py, pz, &s);
    out[0] = s.S; out[1] = s.kbar; out[2] = s.alpha; out[3] = s.vlos; out[4] = s.nu;
    return 0;
}
