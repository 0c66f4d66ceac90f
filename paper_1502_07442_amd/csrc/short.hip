// Exact short-range force tables of a general pair law.
//
// Paper: Croker, ngravs (CPC), section 2.4.1, Eqs. (8)-(11). The TreePM
// split keeps the part of a law's potential that a Gaussian filter of scale
// r_s removes from the mesh: phi_short = phi - F^-1[phi(k) exp(-k^2 r_s^2)].
// The law enters through phibar(k) = k^2 phi(k), its transform normalised by
// the Newtonian Green's function (smooth where phi(k) is singular).
//
// With phi(k) = int phi(x) exp(-i k.x) d^3x and force factors relative to
// Newton's 1/r^2, the short-range factor at radius r is
//   f_short(r) = f_full(r) + 1/(2 pi^2) int_0^inf phibar(k) exp(-k^2 r_s^2)
//                                      [sin(k r)/k - r cos(k r)] dk,
// the r'-integral of Eq. (10) taken in closed form (int_0^r cos(k r') dr' =
// sin(k r)/k) and the derivative of Eq. (11) under the integral.
//
// Design: the integrand is even in k and decays as a Gaussian, so the
// trapezoid rule on k_m = m dk converges geometrically: its error is the
// aliased image of the r-space integrand at distance 2 pi / dk - r (a
// Gaussian of width ~2 r_s, plus the law's own decay, e.g. exp(-r/lambda)
// for a Yukawa term). The paper instead samples the transform on an r grid
// by FFT and integrates it with a 4-point Newton-Cotes rule; the closed-form
// r-integral removes that quadrature and its error term. One thread per
// (species pair, table radius) sums over k with the weights staged in LDS;
// sin and cos of k_m r advance by rotation and are re-seeded every 64 steps.
#include <cmath>
#include <vector>

#include "ngr_internal.hpp"

namespace ngr {
namespace {

constexpr int kShortThreads = 256;
constexpr int kReseed = 64;

// w[ab][m] = trapezoid weight x dk / (2 pi^2) x phibar_ab(k_m) exp(-(k_m r_s)^2)
__global__ void short_weights(uint32_t pairs, uint32_t nk, double dk, double r_s, const double* __restrict__ phibar,
                              double* __restrict__ w)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint64_t)pairs * nk) return;
    const uint32_t m = (uint32_t)(e % nk);
    const double k = m * dk;
    const double trap = m == 0 ? 0.5 : 1.0;
    w[e] = trap * dk / (2.0 * M_PI * M_PI) * phibar[e] * exp(-(k * r_s) * (k * r_s));
}

// tables[ab][i] = f_full[ab][i] + sum_m w[ab][m] (sin(k_m r_i)/k_m - r_i cos(k_m r_i))
__global__ __launch_bounds__(kShortThreads) void short_sum(uint32_t ntab, uint32_t grid, double r_cut, uint32_t nk,
                                                           double dk, const double* __restrict__ w,
                                                           const double* __restrict__ f_full,
                                                           double* __restrict__ tables)
{
    __shared__ double ws[kShortThreads];
    const uint32_t ab = blockIdx.y;
    const uint32_t i = blockIdx.x * kShortThreads + threadIdx.x;
    const bool live = i < ntab;
    const double r = !live ? 0.0
                     : grid == NGR_GRID_R ? i * (r_cut / (ntab - 1))
                                          : sqrt(i * (r_cut * r_cut / (ntab - 1)));
    double sd, cd;
    sincos(dk * r, &sd, &cd);            // rotation by one k step
    double acc = 0.0;
    const double* wab = w + (uint64_t)ab * nk;
    // every thread of the block runs the same chunks (the bound test is inside)
    for (uint32_t base = 0; base < nk; base += kShortThreads) {
        __syncthreads();
        ws[threadIdx.x] = base + threadIdx.x < nk ? wab[base + threadIdx.x] : 0.0;
        __syncthreads();
        const uint32_t cnt = min((uint32_t)kShortThreads, nk - base);
        double s = 0.0, c = 1.0;
        for (uint32_t q = 0; q < cnt; ++q) {
            const uint32_t m = base + q;
            if (q % kReseed == 0) sincos(m * dk * r, &s, &c);
            if (m > 0) acc = fma(ws[q], s / (m * dk) - r * c, acc);
            const double s2 = fma(s, cd, c * sd);
            c = fma(c, cd, -s * sd);
            s = s2;
        }
    }
    if (live) tables[(uint64_t)ab * ntab + i] = f_full[(uint64_t)ab * ntab + i] + acc;
}

}  // namespace

void short_range_grid(double r_s, double r_cut, double range, uint32_t* nk, double* dk)
{
    // period in r: the cut-off plus 12.5 r_s (the Gaussian image below
    // 1e-16) plus 37 ranges (an exp(-r/range) image below 1e-16); k up to
    // where exp(-k^2 r_s^2) < 1e-17
    const double period = r_cut + 12.5 * r_s + 37.0 * range;
    const double step = 2.0 * M_PI / period;
    const double kmax = std::sqrt(17.0 * std::log(10.0)) / r_s;
    *dk = step;
    *nk = (uint32_t)std::ceil(kmax / step) + 1u;
}

void short_range_tables(Context& ctx, const ngr_short_params& sp, const double* phibar, const double* f_full,
                        double* tables)
{
    const uint32_t pairs = sp.D * sp.D, nk = sp.nk, ntab = sp.ntab;
    const size_t wb = (size_t)pairs * nk * sizeof(double), tb = (size_t)pairs * ntab * sizeof(double);
    unsigned char* block = static_cast<unsigned char*>(ctx.alloc(2 * wb + 2 * tb));
    double* phib = reinterpret_cast<double*>(block);
    double* w = reinterpret_cast<double*>(block + wb);
    double* full = reinterpret_cast<double*>(block + 2 * wb);
    double* out = reinterpret_cast<double*>(block + 2 * wb + tb);
    ctx.to_device(phib, phibar, wb);
    ctx.to_device(full, f_full, tb);
    ctx.stage("short-range tables");
    const uint64_t nw = (uint64_t)pairs * nk;
    hipLaunchKernelGGL(short_weights, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, ctx.stream, pairs, nk, sp.dk,
                       sp.r_s, phib, w);
    LAUNCH_CHECK("short_weights");
    hipLaunchKernelGGL(short_sum, dim3((ntab + kShortThreads - 1) / kShortThreads, pairs), dim3(kShortThreads), 0,
                       ctx.stream, ntab, sp.grid, sp.r_cut, nk, sp.dk, w, full, out);
    LAUNCH_CHECK("short_sum");
    ctx.to_host(tables, out, tb);
    ctx.release(block);
}

}  // namespace ngr
