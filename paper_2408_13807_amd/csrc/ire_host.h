// Host-side table construction shared by the single-model and batched paths
// of libire (FP64 on the host, uploaded as FP32 and FP64 copies).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ire_internal.h"

namespace ire {
namespace host {

constexpr double kH = 6.62607015e-27;   // erg s
constexpr double kKB = 1.380649e-16;    // erg / K
constexpr double kC = 2.99792458e10;    // cm / s
constexpr double kPi = 3.14159265358979323846;

// Planck intensity B_nu(T); 0 for T <= 0 and where exp(h nu / kT) overflows.
inline double planck(double nu, double T) {
    if (!(T > 0.0)) return 0.0;
    const double x = kH * nu / (kKB * T);
    if (x > 700.0) return 0.0;
    return (2.0 * kH / (kC * kC)) * nu * nu * nu / std::expm1(x);
}

// Normalised cumulative sums of q (the last entry exactly 1).
inline void cumulative(const double *q, int K, double *out) {
    double total = 0.0;
    for (int k = 0; k < K; ++k) total += q[k];
    double run = 0.0;
    for (int k = 0; k < K; ++k) {
        run += q[k];
        out[k] = total > 0.0 ? run / total : 1.0;
    }
    out[K - 1] = 1.0;
}

// Trapezoid weights in linear frequency (a single frequency gets weight 1).
inline std::vector<double> quadrature_weights(const std::vector<double> &nu) {
    const int K = (int)nu.size();
    std::vector<double> w(K, 1.0);
    if (K == 1) return w;
    for (int k = 0; k < K; ++k) {
        const double left = k > 0 ? nu[k] - nu[k - 1] : 0.0;
        const double right = k + 1 < K ? nu[k + 1] - nu[k] : 0.0;
        w[k] = 0.5 * (left + right);
    }
    return w;
}

// Dust, temperature and re-emission tables (independent of the cloud geometry).
struct DustTables {
    std::vector<double> w;              // K quadrature weights
    std::vector<DustF> df;
    std::vector<DustD> dd;
    std::vector<double> G, lnG, lnT;    // n_t: emitted power per mass and logs
    std::vector<double> D;              // n_t * K re-emission CDF rows
};

// G(T) = 4 pi sum_k kappa_abs B_k(T) w_k on n_t log-spaced temperatures; row 0
// of D is the CDF of kappa_abs B(T_0) w (absorbed power below the first point),
// row j >= 1 that of kappa_abs [B(T_j) - B(T_{j-1})] w.  Returns "" or an error.
inline std::string build_dust_tables(const std::vector<double> &nu, const std::vector<double> &kabs,
                                     const std::vector<double> &albedo, const std::vector<double> &g,
                                     double t_min, double t_max, int nt, DustTables &out) {
    const int K = (int)nu.size();
    out.w = quadrature_weights(nu);
    out.df.resize(K);
    out.dd.resize(K);
    for (int k = 0; k < K; ++k) {
        const double kA = kabs[k];
        const double kS = kA * albedo[k] / (1.0 - albedo[k]);
        const double inv_kS = kS > 0.0 ? 1.0 / kS : HUGE_VAL;
        out.dd[k] = DustD{kA, kS, 1.0 / kA, inv_kS, g[k], albedo[k], kA + kS, 0.0};
        out.df[k] = DustF{(float)kA, (float)kS, (float)(1.0 / kA), kS > 0.0 ? (float)inv_kS : HUGE_VALF,
                          (float)g[k], (float)albedo[k], (float)(kA + kS), 0.0f};
    }
    out.G.assign(nt, 0.0);
    out.lnG.assign(nt, 0.0);
    out.lnT.assign(nt, 0.0);
    out.D.assign((size_t)nt * K, 0.0);
    std::vector<double> Bprev(K, 0.0), Bcur(K), q(K);
    for (int j = 0; j < nt; ++j) {
        const double T = t_min * std::pow(t_max / t_min, (double)j / (double)(nt - 1));
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            Bcur[k] = planck(nu[k], T);
            acc += kabs[k] * Bcur[k] * out.w[k];
            q[k] = kabs[k] * (Bcur[k] - (j == 0 ? 0.0 : Bprev[k])) * out.w[k];
        }
        out.G[j] = 4.0 * kPi * acc;
        out.lnT[j] = std::log(T);
        out.lnG[j] = std::log(out.G[j]);
        cumulative(q.data(), K, out.D.data() + (size_t)j * K);
        Bprev.swap(Bcur);
    }
    if (!(out.G[0] > 0.0)) return "G(t_min) underflows: raise t_min";
    for (int j = 1; j < nt; ++j)
        if (!(out.G[j] > out.G[j - 1])) return "G(T) is not increasing on the temperature grid";
    return "";
}

// Guide table for the G(T) table (layout in ire_internal.h).  Any start is
// correct for the device's bidirectional scan; a good start makes the scan
// one or two steps.
inline void build_guides(const DustTables &dt, std::vector<unsigned char> &out, float &lg0, float &scale) {
    const int nt = (int)dt.G.size();
    out.assign(guide_bytes(nt), 0);
    auto count_le = [](const double *t, int n, double x) {
        int c = 0;
        while (c < n && t[c] <= x) ++c;
        return c;
    };
    const double l0 = std::log2(dt.G[0]), l1 = std::log2(dt.G[nt - 1]);
    lg0 = (float)l0;
    scale = l1 > l0 ? (float)(nt / (l1 - l0)) : 0.0f;
    uint16_t *gg = reinterpret_cast<uint16_t *>(out.data());
    for (int b = 0; b < nt; ++b) {
        const double edge = std::exp2(l0 + (scale > 0.0f ? b / (double)scale : 0.0));
        gg[b] = (uint16_t)count_le(dt.G.data(), nt, edge);
    }
}

// Shell table of one cloud in units of its outer radius: [an empty cavity
// shell when r_edges[0] > 0], the n shells, and a sentinel beyond the surface
// with infinite density.  invM gets the n reciprocal shell masses.
inline void build_shell_table(const double *r_edges, const double *rho, int n, std::vector<ShellF> &shf,
                              std::vector<ShellD> &shd, std::vector<double> &invM) {
    const double Rout = r_edges[n];
    const int cav = r_edges[0] > 0.0 ? 1 : 0;
    const size_t base_f = shf.size(), base_d = shd.size();
    shf.resize(base_f + n + cav + kSentinels);
    shd.resize(base_d + n + cav + kSentinels);
    if (cav) {
        const double a = r_edges[0] / Rout;
        shd[base_d] = ShellD{0.0, a * a, 0.0, 0.0};
        shf[base_f] = ShellF{0.0f, (float)(a * a), 0.0f, 0.0f};
    }
    for (int i = 0; i < n; ++i) {
        const double a = r_edges[i] / Rout, b = r_edges[i + 1] / Rout;
        const double rh = rho[i] * Rout;
        shd[base_d + cav + i] = ShellD{a * a, b * b, rh, rh > 0.0 ? 1.0 / rh : 0.0};
        shf[base_f + cav + i] = ShellF{(float)(a * a), (float)(b * b), (float)rh, rh > 0.0 ? (float)(1.0 / rh) : 0.0f};
        const double r0 = r_edges[i], r1 = r_edges[i + 1];
        const double M = rho[i] * (4.0 * kPi / 3.0) * (r1 * r1 * r1 - r0 * r0 * r0);
        invM.push_back(M > 0.0 ? 1.0 / M : 0.0);
    }
    // the outermost edge is exactly 1 in both precisions
    shd[base_d + cav + n - 1].r2_out = 1.0;
    shf[base_f + cav + n - 1].r2_out = 1.0f;
    for (int j = 0; j < kSentinels; ++j) {
        shd[base_d + cav + n + j] = ShellD{1.0, 4.0, HUGE_VAL, 0.0};
        shf[base_f + cav + n + j] = ShellF{1.0f, 4.0f, HUGE_VALF, 0.0f};
    }
}

// Density-dependent absorption scaling (Sect. 3.2): per record of a shell
// table built by build_shell_table, {k rho, 1/(k rho)} in the same units, with
// k linear in log rho from k_lowest at the lowest density of the model to
// k_highest at the highest (k_highest when all densities are equal); the
// cavity has zero density, the sentinels infinite density.
inline void build_absorption_scaling(const double *r_edges, const double *rho, int n, double k_lowest,
                                     double k_highest, std::vector<float2> &rkf, std::vector<double2> &rkd) {
    const double Rout = r_edges[n];
    const int cav = r_edges[0] > 0.0 ? 1 : 0;
    double lo = HUGE_VAL, hi = -HUGE_VAL;
    for (int i = 0; i < n; ++i)
        if (rho[i] > 0.0) { lo = std::min(lo, std::log(rho[i])); hi = std::max(hi, std::log(rho[i])); }
    rkf.assign((size_t)n + cav + kSentinels, float2{0.0f, 0.0f});
    rkd.assign((size_t)n + cav + kSentinels, double2{0.0, 0.0});
    for (int i = 0; i < n; ++i) {
        double k = k_highest;
        if (rho[i] > 0.0 && hi > lo) k = k_lowest + (k_highest - k_lowest) * (std::log(rho[i]) - lo) / (hi - lo);
        const double ra = k * rho[i] * Rout;
        rkd[cav + i] = double2{ra, ra > 0.0 ? 1.0 / ra : 0.0};
        rkf[cav + i] = float2{(float)ra, ra > 0.0 ? (float)(1.0 / ra) : 0.0f};
    }
    for (int j = 0; j < kSentinels; ++j) {
        rkd[cav + n + j] = double2{HUGE_VAL, 0.0};
        rkf[cav + n + j] = float2{HUGE_VALF, 0.0f};
    }
}

// Device buffer that grows on demand.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    hipError_t upload(const std::vector<T> &h) {
        hipError_t e = ensure(h.size());
        if (e != hipSuccess) return e;
        return hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

inline bool finite_all(const double *a, size_t n) {
    for (size_t j = 0; j < n; ++j)
        if (!std::isfinite(a[j])) return false;
    return true;
}

// Argument checks shared by the single-model and batched setters; "" = valid.
// Weighted-sampling options (Table 1): "" or what is wrong.
inline std::string check_weights(int use_g_E, double g_E, int use_g_S, double g_S, double k_A, double k_S) {
    if ((use_g_E != 0 && use_g_E != 1) || (use_g_S != 0 && use_g_S != 1)) return "use_g_E and use_g_S must be 0 or 1";
    if (!(std::fabs(g_E) < 1.0) || !(std::fabs(g_S) < 1.0)) return "g_E and g_S must be in (-1, 1)";
    if (!(k_A > 0.0) || !(k_S > 0.0) || !std::isfinite(k_A) || !std::isfinite(k_S)) return "k_A and k_S must be finite and > 0";
    return "";
}

inline std::string check_dust(int K, const double *nu, const double *kabs, const double *albedo, const double *g) {
    if (K < 1 || K > kMaxK || !nu || !kabs || !albedo || !g) return "need 1 <= K <= 255 and all dust arrays";
    if (!finite_all(nu, K) || !finite_all(kabs, K) || !finite_all(albedo, K) || !finite_all(g, K))
        return "non-finite dust data";
    for (int k = 0; k < K; ++k) {
        if (!(nu[k] > 0.0) || (k > 0 && !(nu[k] > nu[k - 1]))) return "nu must be positive and increase strictly";
        if (!(kabs[k] > 0.0)) return "kappa_abs must be > 0";
        if (!(albedo[k] >= 0.0 && albedo[k] < 1.0)) return "albedo must be in [0,1)";
        if (!(g[k] > -1.0 && g[k] < 1.0)) return "g must be in (-1,1)";
    }
    return "";
}

inline std::string check_shells(int n, const double *r_edges, const double *rho) {
    if (n < 1 || !r_edges || !rho) return "need n >= 1 shells and both arrays";
    if (!finite_all(r_edges, n + 1) || !finite_all(rho, n)) return "non-finite shell data";
    if (!(r_edges[0] >= 0.0)) return "r_edges[0] must be >= 0";
    for (int i = 0; i < n; ++i) {
        if (!(r_edges[i + 1] > r_edges[i])) return "r_edges must increase strictly";
        if (!(rho[i] >= 0.0)) return "rho must be >= 0";
    }
    return "";
}

}  // namespace host
}  // namespace ire
