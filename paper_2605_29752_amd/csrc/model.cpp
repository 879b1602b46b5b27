// First-principles GEMM landscape and Kernel Optimality Levels (paper Sec. 9 and Sec. 10): the
// ideal ceiling, the optimal achievable landscape from datasheet integers (wave quantization
// over the compute units, memory roofline), and the (tau, rho, level) grade of a measured
// landscape against it.  Also the four-surface decomposition of measured times (Sec. 4).
// Host code only.
#include <algorithm>
#include <cmath>
#include <limits>

#include "sg_internal.h"

namespace {

bool hw_ok(const sg_hw* hw) {
    return hw && hw->peak_tflops > 0.0 && hw->cores > 0 && hw->bw_gbs > 0.0;
}

bool grid_ok(const sg_grid* g) {
    return g && g->step > 0 && g->n_m > 0 && g->n_n > 0 && g->n_k > 0;
}

double ceil_div(double a, double b) { return std::ceil(a / b); }

// Fraction of the launched core-slots that hold work: W / (ceil(W / C) C).
double wave_efficiency(double M, double N, int tile, int cores) {
    const double W = ceil_div(M, tile) * ceil_div(N, tile);
    return W / (ceil_div(W, cores) * cores);
}

// Mean |difference| of consecutive entries along N, averaged over every line along N.
double roughness_n(const double* T, int nm, int nn, int nk) {
    double s = 0.0;
    for (int m = 0; m < nm; ++m)
        for (int k = 0; k < nk; ++k) {
            double line = 0.0;
            for (int n = 0; n + 1 < nn; ++n)
                line += std::fabs(T[((int64_t)m * nn + n + 1) * nk + k] - T[((int64_t)m * nn + n) * nk + k]);
            s += line / (nn - 1);
        }
    return s / ((double)nm * nk);
}

// Channel share of a tensor moved in rows of 256 elements (Sec. 9.2): the address space is
// striped over `channels` channels in `interleave`-byte blocks; a row spans
// w = min(channels, 256 e / interleave) channels and row starts advance by
// s = (L e / interleave) mod channels blocks, reaching channels / gcd(s, channels) of them.
double channel_share(int64_t L, int e, int channels, int interleave) {
    const int64_t w = std::min<int64_t>(channels, std::max<int64_t>(1, (256 * (int64_t)e) / interleave));
    const int64_t s = ((L * e) / interleave) % channels;
    int64_t a = s, b = channels;
    while (b) { const int64_t t = a % b; a = b; b = t; }      // gcd(s, channels)
    return (double)std::min<int64_t>(channels, w * channels / a) / channels;
}

int throughput_band(double tau) { return tau >= 0.95 ? 3 : tau >= 0.75 ? 2 : tau >= 0.50 ? 1 : 0; }
int smoothness_band(double rho) { return rho <= 1.25 ? 3 : rho <= 2.0 ? 2 : rho <= 3.0 ? 1 : 0; }

}  // namespace

extern "C" {

int sg_ideal_landscape(const sg_grid* g, const sg_hw* hw, int tile, double* out) {
    if (!grid_ok(g) || !hw_ok(hw) || tile <= 0 || !out) return sg::fail(SG_EINVAL, "sg_ideal_landscape: bad argument");
    int64_t i = 0;
    for (int a = 0; a < g->n_m; ++a)
        for (int b = 0; b < g->n_n; ++b)
            for (int c = 0; c < g->n_k; ++c) {
                const double M = (double)(a + 1) * g->step, N = (double)(b + 1) * g->step;
                const double W = ceil_div(M, tile) * ceil_div(N, tile);
                out[i++] = hw->peak_tflops * std::min(1.0, W / hw->cores);
            }
    return SG_OK;
}

int sg_optimal_landscape(const sg_grid* g, const sg_hw* hw, const int* tiles, int ntiles, int c_bytes,
                         double* out) {
    return sg_optimal_landscape_ch(g, hw, tiles, ntiles, c_bytes, 0, 256, out);
}

int sg_optimal_landscape_ch(const sg_grid* g, const sg_hw* hw, const int* tiles, int ntiles, int c_bytes,
                            int channels, int interleave, double* out) {
    if (!grid_ok(g) || !hw_ok(hw) || !tiles || ntiles <= 0 || c_bytes <= 0 || !out || channels < 0 ||
        (channels > 0 && interleave <= 0))
        return sg::fail(SG_EINVAL, "sg_optimal_landscape: bad argument");
    for (int t = 0; t < ntiles; ++t)
        if (tiles[t] <= 0) return sg::fail(SG_EINVAL, "sg_optimal_landscape: tile edge must be positive");
    const double peak = hw->peak_tflops * 1e12, bw = hw->bw_gbs * 1e9;
    int64_t i = 0;
    for (int a = 0; a < g->n_m; ++a)
        for (int b = 0; b < g->n_n; ++b)
            for (int c = 0; c < g->n_k; ++c) {
                const double M = (double)(a + 1) * g->step, N = (double)(b + 1) * g->step;
                const double K = (double)(c + 1) * g->step;
                const double flop = 2.0 * M * N * K;
                double ea = 1.0, eb = 1.0, ed = 1.0;
                if (channels > 0) {
                    ea = channel_share((int64_t)K, 2, channels, interleave);
                    eb = channel_share((int64_t)N, 2, channels, interleave);
                    ed = channel_share((int64_t)N, c_bytes, channels, interleave);
                }
                const double t_mem = (2.0 * M * K / ea + 2.0 * K * N / eb + (double)c_bytes * M * N / ed) / bw;
                double best = std::numeric_limits<double>::infinity();
                for (int t = 0; t < ntiles; ++t) {
                    const double t_comp = flop / (peak * wave_efficiency(M, N, tiles[t], hw->cores));
                    best = std::min(best, std::max(t_comp, t_mem));
                }
                out[i++] = flop / best / 1e12;
            }
    return SG_OK;
}

int sg_kol_grade(const double* actual, const double* optimal, int nm, int nn, int nk, sg_kol* out) {
    if (!actual || !optimal || !out || nm < 1 || nn < 2 || nk < 1)
        return sg::fail(SG_EINVAL, "sg_kol_grade: bad argument (n_n must be >= 2)");
    const int64_t total = (int64_t)nm * nn * nk;
    double sa = 0.0, so = 0.0;
    for (int64_t i = 0; i < total; ++i) {
        sa += actual[i];
        so += optimal[i];
    }
    const double ro = roughness_n(optimal, nm, nn, nk);
    if (so <= 0.0 || ro <= 0.0) return sg::fail(SG_EINVAL, "sg_kol_grade: optimal landscape has no mean or no roughness");
    out->tau = sa / so;
    out->rho = roughness_n(actual, nm, nn, nk) / ro;
    out->t_band = throughput_band(out->tau);
    out->s_band = smoothness_band(out->rho);
    out->level = std::min(out->t_band, out->s_band);
    return SG_OK;
}

int sg_decompose(const sg_shape* shapes, int64_t n, const double* t_gemm, const double* t_memory,
                 const sg_hw* hw, int c_bytes, double* t_compute, double* t_overhead,
                 sg_decomp* out) {
    if (!shapes || n <= 0 || !t_gemm || !t_memory || !out || !hw || !(hw->peak_tflops > 0.0) ||
        !(hw->bw_gbs > 0.0) || c_bytes <= 0)
        return sg::fail(SG_EINVAL, "sg_decompose: bad argument");
    const double peak = hw->peak_tflops * 1e12, bw = hw->bw_gbs * 1e9;
    double share = 0.0;
    int64_t cb_bw = 0, cb_meas = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double M = (double)shapes[i].M, N = (double)shapes[i].N, K = (double)shapes[i].K;
        if (!(M > 0 && N > 0 && K > 0) || !(t_gemm[i] > 0.0))
            return sg::fail(SG_EINVAL, "sg_decompose: empty shape or non-positive GEMM time");
        const double tc = 2.0 * M * N * K / peak;
        const double to = t_gemm[i] - std::max(tc, t_memory[i]);
        if (t_compute) t_compute[i] = tc;
        if (t_overhead) t_overhead[i] = to;
        share += to / t_gemm[i];
        if (tc >= (2.0 * M * K + 2.0 * K * N + (double)c_bytes * M * N) / bw) ++cb_bw;
        if (tc >= t_memory[i]) ++cb_meas;
    }
    out->overhead_share = share / (double)n;
    out->cb_bandwidth = (double)cb_bw / (double)n;
    out->cb_measured = (double)cb_meas / (double)n;
    return SG_OK;
}

}  // extern "C"
