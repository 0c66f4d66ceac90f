// Particle-mesh long-range force of D species (the PM half of TreePM).
//
// Paper: Croker, ngravs (CPC). Section 2: PM forces assign particle masses
// to a density on a regular grid, Fourier transform it, multiply by the
// k-space Green's function, transform back and interpolate the resulting
// potential's forces to the particles; in TreePM mode the Green's function
// carries the Gaussian filter exp(-k^2 r_s^2) (section 2.4.1). Section 2.4:
// every species is both a passive and an active mass, so the mesh sees D^2
// species pairs. The assignment, window correction and difference stencil
// are those of the code the paper extends (GADGET-2): cloud in cell, the
// window divided out twice, a 4-point centred difference.
//
// Design (one GPU, HBM-resident meshes):
// - The particles come from a built tree: sorted by species, then along the
//   Morton curve, so each species is one contiguous run and consecutive
//   threads deposit into neighbouring cells.
// - Two real species densities share one complex mesh (real and imaginary
//   parts); ceil(D/2) forward 3-D FFTs replace D. After the transform the two
//   spectra are separated with Z(k) and conj Z(-k).
// - The k-space step handles k and -k in one thread, so it can overwrite the
//   density spectra with the potential spectra in place. Linearity lets it
//   sum the D source species for each sink species before the inverse
//   transform: ceil(D/2) inverse FFTs instead of the D^2 mesh passes the
//   paper's MPI slab decomposition needs. The sink species' real potentials
//   are paired into complex meshes the same way.
// - 3-D FFTs are passes of batched 1-D radix-2 transforms along one axis
//   each, a tile of lines held in LDS per workgroup, three stages at a time
//   in registers between LDS exchanges, the twiddles staged in LDS from a
//   float64 table computed on the host. The x and y passes take tiles of
//   lines adjacent in z, so that the strided axes read contiguous runs. The
//   z transforms of both directions and the k-space step are one pass: a
//   workgroup holds a z line and its mirror line (-x, -y) of every mesh, so
//   both points of every pair (k, -k) are in its LDS. A force is then five
//   sweeps over the meshes (x, y, z with the k-space step, y, x), not seven.
// - The Green's function is a table over q = |k|^2 (2 pi / L)^-2 per
//   distinct law: pairs whose phibar tables agree up to a constant factor
//   share one table and keep the factor (times G_ab) as a coefficient; the
//   tables of one q are adjacent, so a mesh point reads one or two cache lines.
// - Interpolation differentiates the potential on the fly at the eight
//   cloud-in-cell corners of each particle and writes the acceleration in
//   input order.
#include <cmath>
#include <vector>

#include "ngr_internal.hpp"

namespace ngr {
namespace {

constexpr size_t kFftTileBytes = 128 * 1024;   // most LDS for one workgroup's lines

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Mesh layout: point (x, y, z) of a mesh at x XS + y N + z, XS = (N + 1) N,
// and mesh g at g N XS. The unused row y = N pads every x plane by N points:
// the N points of a line along x are then (N + 1) N apart rather than N^2 (a
// power of two, 16 MiB at N = 1024, which put them all on one HBM channel).
__host__ __device__ inline uint64_t plane_stride(uint32_t p) { return ((1ull << p) + 1ull) << p; }
__host__ __device__ inline uint64_t mesh_stride(uint32_t p) { return plane_stride(p) << p; }

// Lower grid index and fraction along one axis of a lattice coordinate:
// u = X N 2^-64 exactly (N = 2^p).
__device__ inline void cic_axis(uint64_t X, uint32_t p, uint32_t& i, double& f)
{
    i = (uint32_t)(X >> (64 - p));
    f = (double)(X & ((1ull << (64 - p)) - 1ull)) * exp2(-(double)(64 - p));
}

// Densities of species blockIdx.y (sorted run [seg[b], seg[b+1])) into the
// real (even b) or imaginary (odd b) part of complex mesh b / 2.
__global__ void pm_deposit(uint64_t n, const uint64_t* __restrict__ X, const double* __restrict__ mass,
                           const uint64_t* __restrict__ seg, uint32_t N, uint32_t p, double inv_h3,
                           double* __restrict__ mesh)
{
    const uint32_t b = blockIdx.y;
    const uint64_t s0 = seg[b], s1 = seg[b + 1];
    const uint64_t XS = plane_stride(p);
    double* m = mesh + 2 * mesh_stride(p) * (b / 2) + (b & 1);
    const uint32_t mask = N - 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = s0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s1; i += stride) {
        uint32_t ix, iy, iz;
        double fx, fy, fz;
        cic_axis(X[i], p, ix, fx);
        cic_axis(X[n + i], p, iy, fy);
        cic_axis(X[2 * n + i], p, iz, fz);
        const double w = mass[i] * inv_h3;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t cx = (ix + (c >> 2)) & mask, cy = (iy + ((c >> 1) & 1)) & mask, cz = (iz + (c & 1)) & mask;
            const double wt = w * ((c >> 2) ? fx : 1.0 - fx) * (((c >> 1) & 1) ? fy : 1.0 - fy) * ((c & 1) ? fz : 1.0 - fz);
            unsafeAtomicAdd(m + 2 * ((uint64_t)cx * XS + (uint64_t)cy * N + cz), wt);
        }
    }
}

// Batched 1-D FFTs of length N = 2^p along one axis of ngrid complex meshes
// (point (x, y, z) at x XS + y N + z, XS = (N + 1) N). A workgroup
// transforms a tile of T lines adjacent in z. Radix-2 decimation in frequency
// in place in LDS, natural order in, bit-reversed order read out.
// sign = +1: exp(-2 pi i k n / N) (forward), -1: exp(+2 pi i k n / N)
// (inverse, unnormalised). The LDS holds T lines of N points and the N / 2
// twiddles.
// axis 1: along y (points N apart);
// axis 2: along x (points XS apart).
// The z transforms (contiguous lines) run inside the k-space pass
// (pm_green_z).

__device__ inline uint32_t lds_swizzle(uint32_t i)
{
    // XOR the low three bits of a point's LDS slot with its higher bits:
    // the strided patterns below (lines adjacent in z, sets of stride d,
    // bit-reversed read-out) then spread over the banks
    return i ^ (((i >> 3) ^ (i >> 6) ^ (i >> 9)) & 7u);
}

// F consecutive radix-2 decimation-in-frequency stages s .. s+F-1 of the T
// lines in LDS. Those stages (halves h, h/2, ...) only mix the 2^F points
// first + m d of a block of 2h, d = h >> (F-1), so each thread loads such a
// set into registers, applies the F stages and stores it back.
// Twiddles: the pair (m, m + span) of stage st takes W^((off + j d) 2^(s+st))
// with j = m mod span, off the set's position below d and W the twiddle of
// one index; since d 2^(s+st) = N 2^st / 2^F, that is w0^(2^st) times the
// 2^F-th root of unity of order j 2^st, with w0 = W^(off 2^s): one table
// read per set, two squarings, and roots of unity that are constants.
template <int F>
__device__ inline void fft_stages(double2* __restrict__ sm, const double2* __restrict__ tw, double sign, uint32_t N,
                                  uint32_t p, uint32_t T, uint32_t s)
{
    constexpr uint32_t M = 1u << F;
    // cos and sin of 2 pi q / 8, q = 0 .. 3
    constexpr double kC[4] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440};
    constexpr double kS[4] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440};
    const uint32_t logh = p - s - 1, logd = logh - (F - 1);
    const uint32_t h = 1u << logh, d = 1u << logd;
    const uint32_t logsets = p - F;       // sets per line: N / M
    for (uint32_t j = threadIdx.x; j < (T << logsets); j += blockDim.x) {
        const uint32_t l = j >> logsets, js = j & ((1u << logsets) - 1u);
        // js -> the block of 2h it lies in and the position below d inside it
        const uint32_t blk = js >> logd, off = js & (d - 1u);
        const uint32_t first = blk * 2 * h + off;   // within the line
        double2 v[M];
#pragma unroll
        for (uint32_t m = 0; m < M; ++m) v[m] = sm[lds_swizzle(l * N + first + m * d)];
        double2 w[F];                               // w0^(2^st)
        w[0] = tw[off << s];
#pragma unroll
        for (int st = 1; st < F; ++st) w[st] = cmul(w[st - 1], w[st - 1]);
#pragma unroll
        for (uint32_t st = 0; st < (uint32_t)F; ++st) {
            const uint32_t span = M >> (st + 1);          // partner distance in m
#pragma unroll
            for (uint32_t m = 0; m < M; ++m) {
                if (m & span) continue;
                const uint32_t q = ((m & (span - 1u)) << st) * (8u / M);   // root angle in 2 pi / 8
                double2 t = w[st];
                if (q) t = cmul(t, make_double2(kC[q], -sign * kS[q]));
                const double2 a = v[m], b = v[m + span];
                v[m] = cadd(a, b);
                v[m + span] = cmul(csub(a, b), t);
            }
        }
#pragma unroll
        for (uint32_t m = 0; m < M; ++m) sm[lds_swizzle(l * N + first + m * d)] = v[m];
    }
}

// One tile's element e (0 .. T N - 1) of a thread: its line l and point k.
// Consecutive threads take the same point of adjacent lines (adjacent in
// memory), so a wave reads runs of T elements.
__device__ __forceinline__ void tile_element(uint32_t e, uint32_t T, uint32_t logT, uint32_t& l, uint32_t& k)
{
    l = e & (T - 1);
    k = e >> logT;
}

// First element of line 0 of tile it (tiles counted over all meshes; N^2 / T
// tiles per mesh).
template <int AXIS>
__device__ __forceinline__ uint64_t tile_origin(uint64_t it, uint32_t p, uint32_t logT)
{
    const uint32_t lt = 2 * p - logT;     // log2 of the tiles per mesh
    const uint64_t tile = it & ((1ull << lt) - 1ull), g = it >> lt;
    const uint64_t N = 1ull << p;
    uint64_t l0;
    if (AXIS == 1) {
        const uint64_t line0 = tile << logT;   // T consecutive lines in the (x, z) plane, z fastest
        const uint64_t x = line0 >> p, z = line0 & (N - 1);
        l0 = x * plane_stride(p) + z;
    } else {
        // T lines adjacent in z at one y; consecutive tiles step y first, so
        // the workgroups running at once read rows of many different y (16
        // KiB apart at N = 1024) in every x plane rather than the same few
        const uint64_t y = tile & (N - 1), z = (tile >> p) << logT;
        l0 = (y << p) + z;
    }
    return g * mesh_stride(p) + l0;
}

// The real and imaginary parts go to separate register arrays: an array of
// double2 held across the tile loop is kept in scratch memory by the compiler.
template <uint32_t EPT, uint32_t NT, int AXIS>
__device__ __forceinline__ void load_tile(double (&rx)[EPT], double (&ry)[EPT], const double2* __restrict__ src,
                                          uint32_t p, uint32_t T, uint32_t logT, uint64_t lstep, uint64_t stride)
{
#pragma unroll
    for (uint32_t i = 0; i < EPT; ++i) {
        uint32_t l, k;
        tile_element(threadIdx.x + i * NT, T, logT, l, k);
        const double2 v = src[l * lstep + k * stride];
        rx[i] = v.x;
        ry[i] = v.y;
    }
}

// EPT = T N / NT elements per thread (NT threads), fixed at compile time so that
// a tile's loads are all issued before the first is waited for. The axis is a
// template parameter too: with it a runtime argument, the gfx950 backend
// (ROCm 7.2) left the register holding log2 T unset on the x-axis path into
// the tile loop, so the x transform read and wrote wrong tiles. A bounded
// grid of workgroups takes tiles in turn; the next tile's loads are issued
// into registers before the current tile's stages, so they are in flight
// while the stages run.
template <uint32_t EPT, uint32_t NT, int AXIS>
__global__ __launch_bounds__(NT) void fft_lines(double2* __restrict__ data, uint32_t N, uint32_t p, uint32_t T,
                                                uint32_t logT, const double2* __restrict__ twiddle, double sign,
                                                uint64_t ntiles)
{
    HIP_DYNAMIC_SHARED(double2, sm);
    double2* tw = sm + (size_t)T * N;     // N / 2 twiddles, conjugated for the inverse (sign -1)
    for (uint32_t k = threadIdx.x; k < N / 2; k += blockDim.x) {
        const double2 w = twiddle[k];
        tw[k] = make_double2(w.x, sign * w.y);
    }
    // distance between a tile's lines and between a line's points
    const uint64_t lstep = 1, stride = AXIS == 1 ? (uint64_t)N : plane_stride(p);
    double rx[EPT], ry[EPT];
    uint64_t it = blockIdx.x;
    if (it < ntiles) load_tile<EPT, NT, AXIS>(rx, ry, data + tile_origin<AXIS>(it, p, logT), p, T, logT, lstep, stride);
    // the trip count is uniform per workgroup
    for (; it < ntiles; it += gridDim.x) {
        __syncthreads();                  // the previous tile's read-out is done (and the twiddles are in)
#pragma unroll
        for (uint32_t i = 0; i < EPT; ++i) {
            uint32_t l, k;
            tile_element(threadIdx.x + i * NT, T, logT, l, k);
            sm[lds_swizzle(l * N + k)] = make_double2(rx[i], ry[i]);
        }
        __syncthreads();
        const uint64_t nx = it + gridDim.x;
        if (nx < ntiles) load_tile<EPT, NT, AXIS>(rx, ry, data + tile_origin<AXIS>(nx, p, logT), p, T, logT, lstep, stride);
        // Radix-2 decimation in frequency, up to three stages per pass held in
        // registers (fft_stages); a barrier between passes.
        for (uint32_t s = 0; s < p;) {
            const uint32_t f = min(3u, p - s);
            if (f == 3) fft_stages<3>(sm, tw, sign, N, p, T, s);
            else if (f == 2) fft_stages<2>(sm, tw, sign, N, p, T, s);
            else fft_stages<1>(sm, tw, sign, N, p, T, s);
            __syncthreads();
            s += f;
        }
        double2* dst = data + tile_origin<AXIS>(it, p, logT);
#pragma unroll
        for (uint32_t i = 0; i < EPT; ++i) {
            uint32_t l, k;
            tile_element(threadIdx.x + i * NT, T, logT, l, k);
            const uint32_t rk = __brev(k) >> (32 - p);
            dst[l * lstep + k * stride] = sm[lds_swizzle(l * N + rk)];
        }
    }
}

// Per species pair: its coefficient and which unique table it scales.
struct PairMix {
    double coef[NGR_MAX_SPECIES * NGR_MAX_SPECIES];
    uint32_t table[NGR_MAX_SPECIES * NGR_MAX_SPECIES];
};

// The k-space step at one pair of points (k, -k): Z[g] = Z_g(k) and Zm[g] =
// Z_g(-k) of the packed meshes in; the packed potential spectra P_g(k) and
// P_g(-k) out. Unpacks the density spectra of every species, forms every sink
// species' potential spectrum sum_b coef_ab u_t(ab)(q) / W(k)^2 rho_b(k), and
// packs the potentials two per mesh. gq[q][t] holds the U unique laws
// phibar_t(q) exp(-k^2 r_s^2) / (k^2 N^3) (0 at q = 0); iw2 = 1 / W(k)^2.
template <uint32_t D>
__device__ __forceinline__ void green_point(double2 (&Z)[(D + 1) / 2], double2 (&Zm)[(D + 1) / 2],
                                            const double* __restrict__ gqq, uint32_t U, double iw2,
                                            const PairMix& mix)
{
    constexpr uint32_t ngrid = (D + 1) / 2;
    double2 rho[2 * ngrid];
#pragma unroll
    for (uint32_t g2 = 0; g2 < ngrid; ++g2) {
        const double2 z = Z[g2], zm = Zm[g2];
        // rho_even(k) = (Z(k) + conj Z(-k)) / 2, rho_odd(k) = (Z(k) - conj Z(-k)) / 2i
        rho[2 * g2] = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
        rho[2 * g2 + 1] = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
    }
    double2 ph[2 * ngrid];
#pragma unroll
    for (uint32_t a = 0; a < 2 * ngrid; ++a) ph[a] = make_double2(0.0, 0.0);
    // Each unique table is read once per point (a lane's q is its own, so a
    // read touches one cache line per lane); the pairs that scale it are
    // selected by the uniform table index.
    for (uint32_t t = 0; t < U; ++t) {
        const double g = gqq[t] * iw2;
#pragma unroll
        for (uint32_t a = 0; a < D; ++a) {
#pragma unroll
            for (uint32_t b = 0; b < D; ++b) {
                if (mix.table[a * D + b] != t) continue;
                const double f = mix.coef[a * D + b] * g;
                ph[a].x = fma(f, rho[b].x, ph[a].x);
                ph[a].y = fma(f, rho[b].y, ph[a].y);
            }
        }
    }
#pragma unroll
    for (uint32_t g2 = 0; g2 < ngrid; ++g2) {
        // P(k) = Phi_even(k) + i Phi_odd(k); P(-k) = conj Phi_even(k) + i conj Phi_odd(k)
        const double2 pe = ph[2 * g2], po = ph[2 * g2 + 1];
        Z[g2] = make_double2(pe.x - po.y, pe.y + po.x);
        Zm[g2] = make_double2(pe.x + po.y, -pe.y + po.x);
    }
}

// Lines along z come in mirror pairs: line (x, y) holds the points (x, y, k),
// line (-x, -y) the points -(x, y, k) up to the sign of k. Pair P (of N^2 / 2
// + 2) is the line with the smaller index: x in 1 .. N/2 - 1 with any y, then
// x = 0 and x = N/2 with y in 0 .. N/2 (four lines are their own mirror).
__device__ __forceinline__ void mirror_pair(uint64_t P, uint32_t p, uint32_t& x, uint32_t& y)
{
    const uint32_t N = 1u << p;
    const uint64_t inner = (uint64_t)(N / 2 - 1) << p;
    if (P < inner) {
        x = 1u + (uint32_t)(P >> p);
        y = (uint32_t)P & (N - 1u);
    } else {
        const uint32_t r = (uint32_t)(P - inner);
        x = r < N / 2 + 1 ? 0u : N / 2;
        y = r < N / 2 + 1 ? r : r - (N / 2 + 1);
    }
}

constexpr uint32_t kFusedThreads = 512;

// The z transforms and the k-space step in one pass. A workgroup takes a
// mirror pair of z lines in every packed mesh (2 ceil(D/2) lines in LDS: slot
// 2g the line (x, y) of mesh g, slot 2g + 1 the mirror line): forward
// transform along z, the k-space step at (k, -k) with both points in LDS,
// inverse transform, write back. The x and y transforms of both directions
// run before and after it, so each mesh is read and written once here where
// separate passes would take three sweeps. The forward output is in
// bit-reversed order; the k-space step reads it there and writes the inverse
// transform's input in natural order (results held in registers across a
// barrier). The next pair's loads are in flight while a pair is transformed.
template <uint32_t D>
__global__ __launch_bounds__(kFusedThreads) void pm_green_z(double2* __restrict__ mesh, uint32_t p, uint32_t U,
                                                            const double* __restrict__ gq,
                                                            const double* __restrict__ s2,
                                                            const double2* __restrict__ twiddle, PairMix mix,
                                                            uint64_t npairs)
{
    constexpr uint32_t ngrid = (D + 1) / 2, L = 2 * ngrid, NT = kFusedThreads;
    constexpr uint32_t EMAX = (L * 1024 + NT - 1) / NT;   // elements per thread at N = 1024
    constexpr uint32_t KMAX = (1024 + NT - 1) / NT;       // points per thread in the k-space step
    const uint32_t N = 1u << p, m = N - 1u, LN = L * N;
    const uint64_t MS = mesh_stride(p), XS = plane_stride(p);
    HIP_DYNAMIC_SHARED(double2, sm);
    double2* twf = sm + (size_t)LN;       // forward twiddles
    double2* twi = twf + N / 2;           // conjugated, for the inverse
    for (uint32_t k = threadIdx.x; k < N / 2; k += NT) {
        const double2 w = twiddle[k];
        twf[k] = w;
        twi[k] = make_double2(w.x, -w.y);
    }
    // the trip count is uniform per workgroup; every workgroup has a first pair
    // (the grid is at most npairs)
    uint64_t P = blockIdx.x;
    uint32_t x, y;
    mirror_pair(P, p, x, y);
    double rx[EMAX], ry[EMAX];
    {
        const uint64_t la = x * XS + ((uint64_t)y << p), lb = ((N - x) & m) * XS + ((uint64_t)((N - y) & m) << p);
#pragma unroll
        for (uint32_t i = 0; i < EMAX; ++i) {
            const uint32_t e = threadIdx.x + i * NT;
            if (e < LN) {
                const uint32_t l = e >> p, k = e & m;
                const double2 v = mesh[(l >> 1) * MS + ((l & 1) ? lb : la) + k];
                rx[i] = v.x;
                ry[i] = v.y;
            }
        }
    }
    for (;;) {
        const uint32_t mx = (N - x) & m, my = (N - y) & m;
        const bool self = mx == x && my == y;
        const uint64_t la = x * XS + ((uint64_t)y << p), lb = mx * XS + ((uint64_t)my << p);
        __syncthreads();                  // the previous pair's read-out is done (and the twiddles are in)
#pragma unroll
        for (uint32_t i = 0; i < EMAX; ++i) {
            const uint32_t e = threadIdx.x + i * NT;
            if (e < LN) sm[lds_swizzle(e)] = make_double2(rx[i], ry[i]);
        }
        __syncthreads();
        const uint64_t nP = P + gridDim.x;
        const bool more = nP < npairs;
        uint32_t nx, ny;
        mirror_pair(more ? nP : P, p, nx, ny);
        if (more) {
            const uint64_t na = nx * XS + ((uint64_t)ny << p),
                           nb = ((N - nx) & m) * XS + ((uint64_t)((N - ny) & m) << p);
#pragma unroll
            for (uint32_t i = 0; i < EMAX; ++i) {
                const uint32_t e = threadIdx.x + i * NT;
                if (e < LN) {
                    const uint32_t l = e >> p, k = e & m;
                    const double2 v = mesh[(l >> 1) * MS + ((l & 1) ? nb : na) + k];
                    rx[i] = v.x;
                    ry[i] = v.y;
                }
            }
        }
        for (uint32_t s = 0; s < p;) {
            const uint32_t f = min(3u, p - s);
            if (f == 3) fft_stages<3>(sm, twf, 1.0, N, p, L, s);
            else if (f == 2) fft_stages<2>(sm, twf, 1.0, N, p, L, s);
            else fft_stages<1>(sm, twf, 1.0, N, p, L, s);
            __syncthreads();
            s += f;
        }
        // k-space step: point k of line (x, y) pairs with point -k of the mirror line
        const int nxs = x < N / 2 ? (int)x : (int)x - (int)N, nys = y < N / 2 ? (int)y : (int)y - (int)N;
        const double wxy = s2[x] * s2[y];
        double2 outA[KMAX][ngrid], outB[KMAX][ngrid];
#pragma unroll
        for (uint32_t j = 0; j < KMAX; ++j) {
            const uint32_t k = threadIdx.x + j * NT;
            if (k < N) {
                const uint32_t mk = (N - k) & m;
                const uint32_t kr = __brev(k) >> (32 - p), mkr = __brev(mk) >> (32 - p);
                const int nz = k < N / 2 ? (int)k : (int)k - (int)N;
                const uint32_t q = (uint32_t)(nxs * nxs + nys * nys + nz * nz);
                const double W = wxy * s2[k];
                double2 Z[ngrid], Zm[ngrid];
#pragma unroll
                for (uint32_t g2 = 0; g2 < ngrid; ++g2) {
                    Z[g2] = sm[lds_swizzle((2 * g2) * N + kr)];
                    Zm[g2] = sm[lds_swizzle((2 * g2 + 1) * N + mkr)];
                }
                green_point<D>(Z, Zm, gq + (uint64_t)q * U, U, 1.0 / (W * W), mix);
#pragma unroll
                for (uint32_t g2 = 0; g2 < ngrid; ++g2) {
                    outA[j][g2] = Z[g2];
                    outB[j][g2] = Zm[g2];
                }
            }
        }
        __syncthreads();                  // every bit-reversed read is done
#pragma unroll
        for (uint32_t j = 0; j < KMAX; ++j) {
            const uint32_t k = threadIdx.x + j * NT;
            if (k < N) {
                const uint32_t mk = (N - k) & m;
#pragma unroll
                for (uint32_t g2 = 0; g2 < ngrid; ++g2) {
                    sm[lds_swizzle((2 * g2) * N + k)] = outA[j][g2];
                    sm[lds_swizzle((2 * g2 + 1) * N + mk)] = outB[j][g2];
                }
            }
        }
        __syncthreads();
        for (uint32_t s = 0; s < p;) {
            const uint32_t f = min(3u, p - s);
            if (f == 3) fft_stages<3>(sm, twi, -1.0, N, p, L, s);
            else if (f == 2) fft_stages<2>(sm, twi, -1.0, N, p, L, s);
            else fft_stages<1>(sm, twi, -1.0, N, p, L, s);
            __syncthreads();
            s += f;
        }
        // read-out in natural order; a line that is its own mirror is written once
#pragma unroll
        for (uint32_t i = 0; i < EMAX; ++i) {
            const uint32_t e = threadIdx.x + i * NT;
            if (e < LN) {
                const uint32_t l = e >> p, k = e & m;
                if (self && (l & 1)) continue;
                const uint32_t r = __brev(k) >> (32 - p);
                mesh[(l >> 1) * MS + ((l & 1) ? lb : la) + k] = sm[lds_swizzle(l * N + r)];
            }
        }
        if (!more) break;
        P = nP;
        x = nx;
        y = ny;
    }
}

// Accelerations of species blockIdx.y: -grad Phi by the 4-point difference at
// the eight cloud-in-cell corners, interpolated with the same weights.
__global__ void pm_interp(uint64_t n, const uint64_t* __restrict__ X, const uint32_t* __restrict__ perm,
                          const uint64_t* __restrict__ seg, uint32_t N, uint32_t p, double inv_h,
                          const double* __restrict__ mesh, double* __restrict__ acc, uint64_t in_off,
                          int accumulate)
{
    const uint32_t a = blockIdx.y;
    const uint64_t s0 = seg[a], s1 = seg[a + 1];
    const uint64_t XS = plane_stride(p);
    const double* m = mesh + 2 * mesh_stride(p) * (a / 2) + (a & 1);
    const uint32_t mask = N - 1;
    auto P = [&](uint32_t x, uint32_t y, uint32_t z) {
        return m[2 * ((uint64_t)(x & mask) * XS + (uint64_t)(y & mask) * N + (z & mask))];
    };
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = s0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s1; i += stride) {
        uint32_t ix, iy, iz;
        double fx, fy, fz;
        cic_axis(X[i], p, ix, fx);
        cic_axis(X[n + i], p, iy, fy);
        cic_axis(X[2 * n + i], p, iz, fz);
        double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t cx = ix + (c >> 2), cy = iy + ((c >> 1) & 1), cz = iz + (c & 1);
            const double wt = ((c >> 2) ? fx : 1.0 - fx) * (((c >> 1) & 1) ? fy : 1.0 - fy) * ((c & 1) ? fz : 1.0 - fz);
            const double gx = 2.0 / 3.0 * (P(cx + 1, cy, cz) - P(cx - 1, cy, cz)) -
                              1.0 / 12.0 * (P(cx + 2, cy, cz) - P(cx - 2, cy, cz));
            const double gy = 2.0 / 3.0 * (P(cx, cy + 1, cz) - P(cx, cy - 1, cz)) -
                              1.0 / 12.0 * (P(cx, cy + 2, cz) - P(cx, cy - 2, cz));
            const double gz = 2.0 / 3.0 * (P(cx, cy, cz + 1) - P(cx, cy, cz - 1)) -
                              1.0 / 12.0 * (P(cx, cy, cz + 2) - P(cx, cy, cz - 2));
            ax = fma(wt, gx, ax);
            ay = fma(wt, gy, ay);
            az = fma(wt, gz, az);
        }
        const uint64_t o = perm[i] - in_off;
        const double vx = -ax * inv_h, vy = -ay * inv_h, vz = -az * inv_h;
        if (accumulate) {
            acc[o] += vx;
            acc[n + o] += vy;
            acc[2 * n + o] += vz;
        } else {
            acc[o] = vx;
            acc[n + o] = vy;
            acc[2 * n + o] = vz;
        }
    }
}

// gq[q][t] = u_t[q] exp(-k_q^2 r_s^2) / (k_q^2 N^3), k_q^2 = q (2 pi / L)^2; 0 at q = 0.
// The U unique tables of one q are adjacent.
__global__ void pm_green_table(uint32_t U, uint32_t nq, const double* __restrict__ tables, double kunit2,
                               double r_s2, double invN3, double* __restrict__ gq)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint64_t)U * nq) return;
    const uint32_t t = (uint32_t)(e / nq), q = (uint32_t)(e % nq);
    const double k2 = q * kunit2;
    gq[(uint64_t)q * U + t] = q == 0 ? 0.0 : tables[e] * exp(-k2 * r_s2) / k2 * invN3;
}

}  // namespace

PmPlan::~PmPlan() = default;

void pm_create(Context& ctx, const ngr_pm_params& pp, const double* G, const double* phibar, PmPlan& pl)
{
    const uint32_t N = pp.N, D = pp.D;
    pl.N = N;
    pl.D = D;
    pl.p = 0;
    while ((1u << pl.p) < N) ++pl.p;
    pl.box = pp.box;
    pl.r_s = pp.r_s;
    pl.nq = 3u * (N / 2) * (N / 2) + 1u;
    // Laws that are the same table up to a constant factor share one table:
    // pair ab uses coef_ab u_t(ab)(q) with coef_ab = G_ab c_ab (on the
    // benchmark's Newtonian laws every pair shares one table).
    const uint32_t pairs = D * D, nq = pl.nq;
    std::vector<uint32_t> rep;            // first pair of each unique table
    for (uint32_t ab = 0; ab < pairs; ++ab) {
        const double* x = phibar + (size_t)ab * nq;
        uint32_t kmax = 1;
        for (uint32_t q = 1; q < nq; ++q)
            if (std::fabs(x[q]) > std::fabs(x[kmax])) kmax = q;
        const double xmax = std::fabs(x[kmax]);
        bool found = false;
        for (uint32_t t = 0; t < rep.size() && !found; ++t) {
            const double* u = phibar + (size_t)rep[t] * nq;
            if (u[kmax] == 0.0 || xmax == 0.0) continue;
            const double c = x[kmax] / u[kmax];
            bool same = true;
            for (uint32_t q = 1; q < nq && same; ++q) same = std::fabs(x[q] - c * u[q]) <= 1e-15 * xmax;
            if (same) {
                pl.mix_table[ab] = t;
                pl.mix_coef[ab] = G[ab] * c;
                found = true;
            }
        }
        if (!found) {
            pl.mix_table[ab] = (uint32_t)rep.size();
            pl.mix_coef[ab] = G[ab];
            rep.push_back(ab);
        }
    }
    pl.U = (uint32_t)rep.size();
    const size_t gq_bytes = (size_t)pl.U * nq * sizeof(double);
    pl.gq = static_cast<double*>(ctx.alloc(gq_bytes));
    pl.s2 = static_cast<double*>(ctx.alloc(N * sizeof(double)));
    pl.tw = static_cast<double2*>(ctx.alloc((N / 2) * sizeof(double2)));
    pl.mesh = static_cast<double2*>(ctx.alloc((size_t)((D + 1) / 2) * mesh_stride(pl.p) * sizeof(double2)));
    // host tables: sinc^2 per grid index (signed frequency), twiddles exp(-2 pi i m / N)
    std::vector<double> s2(N);
    for (uint32_t i = 0; i < N; ++i) {
        const int ni = i < N / 2 ? (int)i : (int)i - (int)N;
        const double x = M_PI * ni / N;
        const double sn = ni == 0 ? 1.0 : std::sin(x) / x;
        s2[i] = sn * sn;
    }
    std::vector<double2> tw(N / 2);
    for (uint32_t m = 0; m < N / 2; ++m) {
        const double t = -2.0 * M_PI * m / N;
        tw[m] = make_double2(std::cos(t), std::sin(t));
    }
    ctx.to_device(pl.s2, s2.data(), N * sizeof(double));
    ctx.to_device(pl.tw, tw.data(), (N / 2) * sizeof(double2));
    double* stage = static_cast<double*>(ctx.alloc(gq_bytes));
    for (uint32_t t = 0; t < pl.U; ++t)
        ctx.to_device(stage + (size_t)t * nq, phibar + (size_t)rep[t] * nq, nq * sizeof(double));
    const double kunit = 2.0 * M_PI / pp.box;
    const uint64_t ne = (uint64_t)pl.U * nq;
    hipLaunchKernelGGL(pm_green_table, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, ctx.stream, pl.U, nq, stage,
                       kunit * kunit, pp.r_s * pp.r_s, 1.0 / ((double)N * N * N), pl.gq);
    LAUNCH_CHECK("pm_green_table");
    ctx.sync();
    ctx.release(stage);
}

void pm_destroy(Context& ctx, PmPlan& pl)
{
    ctx.release(pl.gq);
    ctx.release(pl.s2);
    ctx.release(pl.tw);
    ctx.release(pl.mesh);
    pl.gq = pl.s2 = nullptr;
    pl.tw = pl.mesh = nullptr;
}

// One pass of 1-D transforms along y (axis 1) or x (axis 2) over every mesh.
static void fft_axis(Context& ctx, PmPlan& pl, uint32_t ngrid, double sign, int axis)
{
    const uint32_t N = pl.N;
    // lines per workgroup (adjacent in z): as many as fit kFftTileBytes, for
    // longer contiguous runs: 8 lines at N = 1024 read whole 128-byte lines of
    // memory (4 lines read half lines)
    const size_t tile_max = std::min(kFftTileBytes, ctx.lds_per_block - (N / 2) * sizeof(double2));
    uint32_t T = 1;
    while (T < 16 && (size_t)(2 * T) * N * sizeof(double2) <= tile_max && 2 * T <= N) T *= 2;
    uint32_t logT = 0;
    while ((1u << logT) < T) ++logT;
    const size_t lds = (size_t)T * N * sizeof(double2) + (N / 2) * sizeof(double2);
    const uint64_t ntiles = (uint64_t)ngrid * ((uint64_t)N * N / T);
    // 256 threads, 512 for tiles over 64 KiB (at most 16 elements a thread)
    const uint32_t NT = (size_t)T * N * sizeof(double2) > 64 * 1024 ? 512 : 256;
    const uint32_t ept = (T * N) / NT;
    if ((T * N) % NT != 0 || ept < 1 || ept > 16 || (ept & (ept - 1)) != 0 || (NT == 512 && ept != 16) ||
        lds > ctx.lds_per_block)
        fail(NGR_EINVAL, "pm: an FFT tile of " + std::to_string(T) + " lines of " + std::to_string(N) +
                             " points does not fit one workgroup");
    // as many workgroups as fit on the device at once (LDS-bound), each looping over tiles
    const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, ctx.lds_per_block / lds));
    const uint64_t blocks = std::min<uint64_t>(ntiles, per_cu * (uint64_t)ctx.num_cu);
    const dim3 grid((unsigned)blocks);
#define NGR_FFT_LAUNCH(E, W)                                                                                        \
    if (axis == 1)                                                                                                   \
        hipLaunchKernelGGL((fft_lines<E, W, 1>), grid, dim3(W), lds, ctx.stream, pl.mesh, N, pl.p, T, logT, pl.tw,  \
                           sign, ntiles);                                                                            \
    else                                                                                                             \
        hipLaunchKernelGGL((fft_lines<E, W, 2>), grid, dim3(W), lds, ctx.stream, pl.mesh, N, pl.p, T, logT, pl.tw,  \
                           sign, ntiles)
    if (NT == 512) {
        NGR_FFT_LAUNCH(16, 512);
    } else {
        switch (ept) {
        case 1: NGR_FFT_LAUNCH(1, 256); break;
        case 2: NGR_FFT_LAUNCH(2, 256); break;
        case 4: NGR_FFT_LAUNCH(4, 256); break;
        case 8: NGR_FFT_LAUNCH(8, 256); break;
        default: NGR_FFT_LAUNCH(16, 256); break;
        }
    }
#undef NGR_FFT_LAUNCH
    LAUNCH_CHECK("fft_lines");
}

// The z transforms of both directions and the k-space step (pm_green_z).
static void green_z(Context& ctx, PmPlan& pl, uint32_t ngrid)
{
    const uint32_t N = pl.N, D = pl.D;
    const size_t lds = (size_t)(2 * ngrid * N + N) * sizeof(double2);
    if (lds > ctx.lds_per_block)
        fail(NGR_EINVAL, "pm: the k-space pass needs " + std::to_string(lds) + " bytes of LDS per workgroup");
    PairMix mix{};
    for (uint32_t ab = 0; ab < D * D; ++ab) {
        mix.coef[ab] = pl.mix_coef[ab];
        mix.table[ab] = pl.mix_table[ab];
    }
    const uint64_t npairs = (uint64_t)N * N / 2 + 2;
    const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(4, ctx.lds_per_block / lds));
    const dim3 grid((unsigned)std::min<uint64_t>(npairs, per_cu * (uint64_t)ctx.num_cu)), block(kFusedThreads);
#define NGR_GZ_LAUNCH(DD)                                                                                            \
    hipLaunchKernelGGL(pm_green_z<DD>, grid, block, lds, ctx.stream, pl.mesh, pl.p, pl.U, pl.gq, pl.s2, pl.tw, mix, \
                       npairs)
    switch (D) {
    case 1: NGR_GZ_LAUNCH(1); break;
    case 2: NGR_GZ_LAUNCH(2); break;
    case 3: NGR_GZ_LAUNCH(3); break;
    case 4: NGR_GZ_LAUNCH(4); break;
    case 5: NGR_GZ_LAUNCH(5); break;
    default: NGR_GZ_LAUNCH(6); break;
    }
#undef NGR_GZ_LAUNCH
    LAUNCH_CHECK("pm_green_z");
}

void pm_force(Context& ctx, PmPlan& pl, const Tree& t, double* acc, int accumulate, PmTimes* times)
{
    const uint32_t N = pl.N, D = pl.D, ngrid = (D + 1) / 2;
    const uint64_t n = t.n;
    const double h = pl.box / N;
    hipEvent_t ev[6];
    for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
    HIP_CHECK(hipEventRecord(ev[0], ctx.stream));
    uint64_t* seg = static_cast<uint64_t*>(ctx.alloc((NGR_MAX_SPECIES + 1) * sizeof(uint64_t)));
    ctx.to_device(seg, t.seg, (NGR_MAX_SPECIES + 1) * sizeof(uint64_t));
    HIP_CHECK(hipMemsetAsync(pl.mesh, 0, (size_t)ngrid * mesh_stride(pl.p) * sizeof(double2), ctx.stream));
    const unsigned gx = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096));
    if (n) {
        hipLaunchKernelGGL(pm_deposit, dim3(gx, D), dim3(256), 0, ctx.stream, n, t.X, t.mass, seg, N, pl.p,
                           1.0 / (h * h * h), reinterpret_cast<double*>(pl.mesh));
        LAUNCH_CHECK("pm_deposit");
    }
    HIP_CHECK(hipEventRecord(ev[1], ctx.stream));
    fft_axis(ctx, pl, ngrid, 1.0, 2);
    fft_axis(ctx, pl, ngrid, 1.0, 1);
    HIP_CHECK(hipEventRecord(ev[2], ctx.stream));
    green_z(ctx, pl, ngrid);
    HIP_CHECK(hipEventRecord(ev[3], ctx.stream));
    fft_axis(ctx, pl, ngrid, -1.0, 1);
    fft_axis(ctx, pl, ngrid, -1.0, 2);
    HIP_CHECK(hipEventRecord(ev[4], ctx.stream));
    if (n) {
        hipLaunchKernelGGL(pm_interp, dim3(gx, D), dim3(256), 0, ctx.stream, n, t.X, t.perm, seg, N, pl.p, 1.0 / h,
                           reinterpret_cast<const double*>(pl.mesh), acc, t.boff[0], accumulate);
        LAUNCH_CHECK("pm_interp");
    }
    HIP_CHECK(hipEventRecord(ev[5], ctx.stream));
    ctx.sync();
    ctx.release(seg);
    if (times) {
        float ms[5];
        for (int k = 0; k < 5; ++k) HIP_CHECK(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
        times->deposit = ms[0];
        times->fft_forward = ms[1];
        times->green = ms[2];
        times->fft_inverse = ms[3];
        times->interp = ms[4];
    }
    for (auto& e : ev) HIP_CHECK(hipEventDestroy(e));
}

}  // namespace ngr
