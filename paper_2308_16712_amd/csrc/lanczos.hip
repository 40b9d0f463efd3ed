// Lanczos ground-state solve on top of the on-the-fly product.
//
// The paper's product is consumed by Krylov eigensolvers that call it
// hundreds to thousands of times (Section 2.1, Section 6.3).  This driver
// keeps every Krylov vector resident in HBM and runs the three-term
// recurrence in FP64:
//   w = H v_k;  alpha_k = Re<v_k, w>;  w -= alpha_k v_k + beta_k v_{k-1};
//   CGS2 (twice: h = V^H w; w -= V h);  beta_{k+1} = ||w||;
//   v_{k+1} = w / beta_{k+1}.
// The second Gram-Schmidt pass is either always run (full CGS2) or run only
// when the first pass removed more than half of ||w||^2 (the test of Daniel,
// Gragg, Kaufman and Stewart, 1976, with eta^2 = 1/2); the decision is taken
// on the device, so the stepper below needs no extra synchronisation.
// Dot products use a fixed grid and a fixed reduction tree, so results do
// not depend on scheduling.  The m x m tridiagonal eigenproblem is solved on
// the host (Sturm-sequence bisection for the lowest eigenvalue, inverse
// iteration for the last component of its eigenvector).

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "ls_internal.hpp"

namespace ls {

namespace {

constexpr int kBlock = 256;
constexpr int kDotBlocks = 2048;   // 8 workgroups per CU: enough loads in flight to stream V
constexpr int kTile = 8;    // Krylov vectors per pass of the multi-dot

template <bool CPLX>
struct V;
template <>
struct V<false> {
    using T = double;
};
template <>
struct V<true> {
    using T = double2;
};

__device__ __forceinline__ double block_reduce(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// partial[b] (re, im) = sum over the block's fixed index set of conj(a) b
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) k_dot_partial(const void *pa, const void *pb, uint64_t n, double2 *partial) {
    __shared__ double sh[kBlock];
    double re = 0.0, im = 0.0;
    const uint64_t stride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        if constexpr (CPLX) {
            const double2 a = static_cast<const double2 *>(pa)[i];
            const double2 b = static_cast<const double2 *>(pb)[i];
            re = fma(a.x, b.x, fma(a.y, b.y, re));
            im = fma(a.x, b.y, fma(-a.y, b.x, im));
        } else {
            re = fma(static_cast<const double *>(pa)[i], static_cast<const double *>(pb)[i], re);
        }
    }
    re = block_reduce(re, sh);
    if constexpr (CPLX) im = block_reduce(im, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(re, im);
}

// out[j] = sum_b partial[b * stride + j], b = 0..nb-1 in a fixed tree
__global__ void __launch_bounds__(kBlock) k_reduce_partials(const double2 *partial, int nb, int stride, double2 *out) {
    __shared__ double sh[kBlock];
    const int j = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        re += partial[static_cast<size_t>(b) * stride + j].x;
        im += partial[static_cast<size_t>(b) * stride + j].y;
    }
    re = block_reduce(re, sh);
    im = block_reduce(im, sh);
    if (threadIdx.x == 0) out[j] = make_double2(re, im);
}

// partial[b][j0 + q] = sum over the block's rows of conj(V_{j0+q}) w, q < tile.
// With wn != null also wn[b] = the block's part of ||w||^2 (accumulated as
// k_dot_partial does).  Does nothing when gate is set and *gate == 0.
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) k_multidot_partial(const void *pV, uint64_t n, int j0, int tile,
                                                             const void *pw, double2 *partial, int stride,
                                                             const int *gate, double2 *wn) {
    if (gate && *gate == 0) return;
    __shared__ double sh[kBlock];
    double re[kTile], im[kTile];
    double nre = 0.0;
#pragma unroll
    for (int q = 0; q < kTile; ++q) re[q] = im[q] = 0.0;
    const uint64_t gstride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += gstride) {
        if constexpr (CPLX) {
            const double2 w = static_cast<const double2 *>(pw)[i];
            if (wn) nre = fma(w.x, w.x, fma(w.y, w.y, nre));
            const double2 *Vb = static_cast<const double2 *>(pV);
#pragma unroll
            for (int q = 0; q < kTile; ++q) {
                if (q < tile) {
                    const double2 v = Vb[static_cast<uint64_t>(j0 + q) * n + i];
                    re[q] = fma(v.x, w.x, fma(v.y, w.y, re[q]));
                    im[q] = fma(v.x, w.y, fma(-v.y, w.x, im[q]));
                }
            }
        } else {
            const double w = static_cast<const double *>(pw)[i];
            if (wn) nre = fma(w, w, nre);
            const double *Vb = static_cast<const double *>(pV);
#pragma unroll
            for (int q = 0; q < kTile; ++q)
                if (q < tile) re[q] = fma(Vb[static_cast<uint64_t>(j0 + q) * n + i], w, re[q]);
        }
    }
    for (int q = 0; q < tile; ++q) {
        const double r = block_reduce(re[q], sh);
        double m = 0.0;
        if constexpr (CPLX) m = block_reduce(im[q], sh);
        if (threadIdx.x == 0) partial[static_cast<size_t>(blockIdx.x) * stride + j0 + q] = make_double2(r, m);
    }
    if (wn) {
        const double r = block_reduce(nre, sh);
        if (threadIdx.x == 0) wn[blockIdx.x] = make_double2(r, 0.0);
    }
}

// w -= sum_j V_j h_j over the rows of the fixed grid of the dot products;
// with wn != null also wn[b] = the block's part of ||w||^2 of the new w (the
// same rows and order as k_dot_partial, so the same value as a separate dot).
// Does nothing when gate is set and *gate == 0.
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) k_gemv_sub(const void *pV, uint64_t n, int nv, const double2 *h, void *pw,
                                                     const int *gate, double2 *wn) {
    if (gate && *gate == 0) return;
    __shared__ double sh[kBlock];
    double nre = 0.0;
    const uint64_t gstride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += gstride) {
        if constexpr (CPLX) {
            const double2 *Vb = static_cast<const double2 *>(pV);
            double2 w = static_cast<double2 *>(pw)[i];
            double sre = 0.0, sim = 0.0;
            for (int j = 0; j < nv; ++j) {
                const double2 v = Vb[static_cast<uint64_t>(j) * n + i];
                const double2 c = h[j];
                sre = fma(v.x, c.x, fma(-v.y, c.y, sre));
                sim = fma(v.x, c.y, fma(v.y, c.x, sim));
            }
            w.x -= sre;
            w.y -= sim;
            static_cast<double2 *>(pw)[i] = w;
            nre = fma(w.x, w.x, fma(w.y, w.y, nre));
        } else {
            const double *Vb = static_cast<const double *>(pV);
            double s = 0.0;
            for (int j = 0; j < nv; ++j) s = fma(Vb[static_cast<uint64_t>(j) * n + i], h[j].x, s);
            const double w = static_cast<double *>(pw)[i] - s;
            static_cast<double *>(pw)[i] = w;
            nre = fma(w, w, nre);
        }
    }
    if (wn) {
        const double r = block_reduce(nre, sh);
        if (threadIdx.x == 0) wn[blockIdx.x] = make_double2(r, 0.0);
    }
}

// Second pass needed (DGKS): ||w1||^2 < ||w||^2 / 2.  nrm = ||w1||^2.
__global__ void k_reorth_decide(const double2 *wn, const double2 *w1n, int *gate, double2 *nrm) {
    *gate = w1n[0].x < 0.5 * wn[0].x ? 1 : 0;
    nrm[0] = w1n[0];
}

// nrm = ||w2||^2 when the second pass ran
__global__ void k_reorth_pick(const int *gate, const double2 *w2n, double2 *nrm) {
    if (*gate) nrm[0] = w2n[0];
}

// w -= alpha v + beta vp   (vp may be null)
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) k_three_term(void *pw, const void *pv, const void *pvp, uint64_t n,
                                                       double alpha, double beta) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    if constexpr (CPLX) {
        double2 w = static_cast<double2 *>(pw)[i];
        const double2 v = static_cast<const double2 *>(pv)[i];
        w.x -= alpha * v.x;
        w.y -= alpha * v.y;
        if (pvp) {
            const double2 u = static_cast<const double2 *>(pvp)[i];
            w.x -= beta * u.x;
            w.y -= beta * u.y;
        }
        static_cast<double2 *>(pw)[i] = w;
    } else {
        double w = static_cast<double *>(pw)[i];
        w -= alpha * static_cast<const double *>(pv)[i];
        if (pvp) w -= beta * static_cast<const double *>(pvp)[i];
        static_cast<double *>(pw)[i] = w;
    }
}

// dst = src / s (element-wise over doubles)
__global__ void __launch_bounds__(kBlock) k_div(double *dst, const double *src, uint64_t n, double s) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i] / s;
}

// Start vector from the counter generator built on the paper's hash64_01.
__device__ __forceinline__ uint64_t mix(uint64_t x) {
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

__global__ void __launch_bounds__(kBlock) k_fill_uniform(double *out, uint64_t count, uint64_t seed) {
    const uint64_t c = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= count) return;
    const uint64_t u = mix(seed + (c + 1) * 0x9E3779B97F4A7C15ULL);
    out[c] = 2.0 * (static_cast<double>(u >> 11) * 0x1.0p-53) - 1.0;
}

uint32_t grid(uint64_t n) { return static_cast<uint32_t>((n + kBlock - 1) / kBlock); }

// Device work buffers of the reorthogonalisation.
struct ReorthBufs {
    double2 *partial;   // [kDotBlocks][m] multi-dot parts (stride m)
    double2 *npart;     // [2][kDotBlocks] block parts of ||w||^2 before / after a pass
    double2 *hs;        // [m] coefficients h = V^H w
    double2 *nrm;       // [4] reduced ||w||^2, ||w1||^2, ||w2||^2; [3] free for the caller
    int *gate;          // second pass needed
    int m;
};

enum { kReorthNone = 0, kReorthFull = 1, kReorthSelective = 2 };

// aux: npart [2][kDotBlocks] | nrm [4] | gate
constexpr size_t kAuxBytes = (2 * kDotBlocks + 4) * sizeof(double2) + 16;
ReorthBufs reorth_bufs(double2 *partial, double2 *hs, void *aux, int m) {
    ReorthBufs b;
    b.partial = partial;
    b.hs = hs;
    b.npart = static_cast<double2 *>(aux);
    b.nrm = b.npart + 2 * kDotBlocks;
    b.gate = reinterpret_cast<int *>(b.nrm + 4);
    b.m = m;
    return b;
}

// Orthogonalises w against V_0 .. V_{nv-1} (mode: none, two passes, or a
// second pass only when the first removed more than half of ||w||^2) and
// leaves ||w||^2 of the result in out[0].x.
template <bool CPLX>
void enqueue_reorth(const void *Vb, uint64_t n, int nv, int mode, void *w, const ReorthBufs &b, double2 *out,
                    hipStream_t st) {
    if (mode == kReorthNone) {
        hipLaunchKernelGGL(k_dot_partial<CPLX>, dim3(kDotBlocks), dim3(kBlock), 0, st, w, w, n, b.partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, b.partial, kDotBlocks, 1, out);
        return;
    }
    const bool sel = mode == kReorthSelective;
    double2 *before = b.npart, *after = b.npart + kDotBlocks;
    for (int pass = 0; pass < 2; ++pass) {
        const int *g = (sel && pass == 1) ? b.gate : nullptr;
        for (int j0 = 0; j0 < nv; j0 += kTile)
            hipLaunchKernelGGL(k_multidot_partial<CPLX>, dim3(kDotBlocks), dim3(kBlock), 0, st, Vb, n, j0,
                               std::min(kTile, nv - j0), w, b.partial, b.m, g,
                               (sel && pass == 0 && j0 == 0) ? before : nullptr);
        hipLaunchKernelGGL(k_reduce_partials, dim3(nv), dim3(kBlock), 0, st, b.partial, kDotBlocks, b.m, b.hs);
        hipLaunchKernelGGL(k_gemv_sub<CPLX>, dim3(kDotBlocks), dim3(kBlock), 0, st, Vb, n, nv, b.hs, w, g,
                           (sel || pass == 1) ? after : nullptr);
        if (sel && pass == 0) {
            hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, before, kDotBlocks, 1, b.nrm);
            hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, after, kDotBlocks, 1, b.nrm + 1);
            hipLaunchKernelGGL(k_reorth_decide, dim3(1), dim3(1), 0, st, b.nrm, b.nrm + 1, b.gate, out);
        }
    }
    if (sel) {
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, after, kDotBlocks, 1, b.nrm + 2);
        hipLaunchKernelGGL(k_reorth_pick, dim3(1), dim3(1), 0, st, b.gate, b.nrm + 2, out);
    } else {
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, after, kDotBlocks, 1, out);
    }
}

// Lowest eigenvalue of the symmetric tridiagonal (a, b) by Sturm bisection.
double tridiag_lowest(const std::vector<double> &a, const std::vector<double> &b) {
    const size_t m = a.size();
    double lo = a[0], hi = a[0];
    for (size_t i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    const double tiny = std::max(scale, 1.0) * 1e-300;
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = a[0] - x;
        if (q < 0) ++cnt;
        for (size_t i = 1; i < m; ++i) {
            if (std::fabs(q) < tiny) q = -tiny;
            q = a[i] - x - b[i - 1] * b[i - 1] / q;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(mid) >= 1) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for eigenvalue theta
double tridiag_last_component(const std::vector<double> &a, const std::vector<double> &b, double theta) {
    const size_t m = a.size();
    if (m == 1) return 1.0;
    double norm_t = 0.0;
    for (size_t i = 0; i < m; ++i) norm_t = std::max(norm_t, std::fabs(a[i]) + (i ? std::fabs(b[i - 1]) : 0.0));
    const double eps = std::max(norm_t, 1.0) * 1e-15;
    std::vector<double> z(m, 1.0), c(m), d(m), rhs(m);
    for (int pass = 0; pass < 3; ++pass) {
        // Thomas solve of (T - theta) y = z with pivot guard
        for (size_t i = 0; i < m; ++i) rhs[i] = z[i];
        d[0] = a[0] - theta;
        if (std::fabs(d[0]) < eps) d[0] = eps;
        for (size_t i = 1; i < m; ++i) {
            const double l = b[i - 1] / d[i - 1];
            d[i] = a[i] - theta - l * b[i - 1];
            if (std::fabs(d[i]) < eps) d[i] = eps;
            rhs[i] -= l * rhs[i - 1];
        }
        z[m - 1] = rhs[m - 1] / d[m - 1];
        for (size_t i = m - 1; i-- > 0;) z[i] = (rhs[i] - b[i] * z[i + 1]) / d[i];
        double nz = 0.0;
        for (double v : z) nz += v * v;
        nz = std::sqrt(nz);
        for (double &v : z) v /= nz;
    }
    return std::fabs(z[m - 1]);
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() { if (p) hipFree(p); }
};

template <bool CPLX>
ls_status lanczos_impl(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t st, double *e0_out,
                       uint32_t *iters_out, double *resid_out) {
    using T = typename V<CPLX>::T;
    const uint64_t n = op->basis->dim;
    const uint32_t m = static_cast<uint32_t>(std::min<uint64_t>(o->max_iter, n));
    const size_t es = sizeof(T);
    DevMem Vm, wm, part, scal, aux;
    hipError_t err = hipMalloc(&Vm.p, static_cast<size_t>(m) * n * es);
    if (err != hipSuccess) throw Error{LS_ENOMEM, "cannot allocate the Krylov vectors"};
    LS_HIP_CHECK(hipMalloc(&wm.p, n * es));
    LS_HIP_CHECK(hipMalloc(&part.p, static_cast<size_t>(kDotBlocks) * std::max<uint32_t>(m, 1) * sizeof(double2)));
    LS_HIP_CHECK(hipMalloc(&scal.p, std::max<uint32_t>(m, 1) * sizeof(double2)));
    LS_HIP_CHECK(hipMalloc(&aux.p, kAuxBytes));
    T *Vb = static_cast<T *>(Vm.p);
    T *w = static_cast<T *>(wm.p);
    double2 *partial = static_cast<double2 *>(part.p);
    double2 *hs = static_cast<double2 *>(scal.p);
    const uint64_t nd = n * (CPLX ? 2 : 1);    // doubles per vector
    const ReorthBufs rb = reorth_bufs(partial, hs, aux.p, static_cast<int>(m));

    auto dot = [&](const T *x, const T *y) {
        hipLaunchKernelGGL(k_dot_partial<CPLX>, dim3(kDotBlocks), dim3(kBlock), 0, st, x, y, n, partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, kDotBlocks, 1, hs);
        double2 r;
        LS_HIP_CHECK(hipMemcpyAsync(&r, hs, sizeof(double2), hipMemcpyDeviceToHost, st));
        LS_HIP_CHECK(hipStreamSynchronize(st));
        return r;
    };

    // start vector
    if (o->d_v0) {
        LS_HIP_CHECK(hipMemcpyAsync(w, o->d_v0, n * es, hipMemcpyDeviceToDevice, st));
    } else {
        hipLaunchKernelGGL(k_fill_uniform, dim3(grid(nd)), dim3(kBlock), 0, st, reinterpret_cast<double *>(w), nd,
                           o->seed);
    }
    LS_HIP_CHECK(hipGetLastError());
    const double nrm0 = std::sqrt(dot(w, w).x);
    if (!(nrm0 > 0.0)) throw Error{LS_EINVAL, "the start vector is zero"};
    hipLaunchKernelGGL(k_div, dim3(grid(nd)), dim3(kBlock), 0, st, reinterpret_cast<double *>(Vb),
                       reinterpret_cast<const double *>(w), nd, nrm0);

    std::vector<double> alpha, beta;
    double e0 = 0.0, resid = INFINITY, prev = 0.0;
    bool have_prev = false, converged = false;
    for (uint32_t k = 0; k < m; ++k) {
        T *vk = Vb + static_cast<uint64_t>(k) * n;
        launch_matvec(op, 1, vk, w, st);
        const double a = dot(vk, w).x;
        hipLaunchKernelGGL(k_three_term<CPLX>, dim3(grid(n)), dim3(kBlock), 0, st, w, vk,
                           k > 0 ? Vb + static_cast<uint64_t>(k - 1) * n : nullptr, n, a,
                           k > 0 ? beta[k - 1] : 0.0);
        enqueue_reorth<CPLX>(Vb, n, static_cast<int>(k) + 1, static_cast<int>(o->reorth), w, rb, rb.nrm + 3, st);
        LS_HIP_CHECK(hipGetLastError());
        double2 wn;
        uint32_t miss = 0;
        LS_HIP_CHECK(hipMemcpyAsync(&wn, rb.nrm + 3, sizeof(double2), hipMemcpyDeviceToHost, st));
        enqueue_flag_read(op, &miss, st);
        LS_HIP_CHECK(hipStreamSynchronize(st));
        if (miss)
            throw Error{LS_EINTERNAL, "Lanczos step " + std::to_string(k) +
                                          ": the product met a neighbour whose representative lies in the sector "
                                          "but is missing from the basis"};
        const double bnext = std::sqrt(wn.x);
        alpha.push_back(a);
        e0 = tridiag_lowest(alpha, beta);
        resid = bnext * tridiag_last_component(alpha, beta, e0);
        const double scale = std::max(1.0, std::fabs(e0));
        if (o->tol > 0 && have_prev && std::fabs(e0 - prev) < o->tol * scale && resid < std::sqrt(o->tol) * scale) {
            converged = true;
            break;
        }
        prev = e0;
        have_prev = true;
        if (k + 1 < m) {
            if (bnext == 0.0) break;
            beta.push_back(bnext);
            hipLaunchKernelGGL(k_div, dim3(grid(nd)), dim3(kBlock), 0, st,
                               reinterpret_cast<double *>(Vb + static_cast<uint64_t>(k + 1) * n),
                               reinterpret_cast<const double *>(w), nd, bnext);
        }
    }
    LS_HIP_CHECK(hipStreamSynchronize(st));
    if (o->alpha)
        for (size_t k = 0; k < alpha.size(); ++k) o->alpha[k] = alpha[k];
    if (o->beta)
        for (size_t k = 0; k < beta.size(); ++k) o->beta[k] = beta[k];
    if (e0_out) *e0_out = e0;
    if (iters_out) *iters_out = static_cast<uint32_t>(alpha.size());
    if (resid_out) *resid_out = resid;
    return (o->tol > 0 && !converged) ? LS_WNOTCONV : LS_OK;
}

}  // namespace

ls_status run_lanczos(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t st, double *e0, uint32_t *iters,
                      double *resid) {
    if (op->is_complex) return lanczos_impl<true>(op, o, st, e0, iters, resid);
    return lanczos_impl<false>(op, o, st, e0, iters, resid);
}

// ---- the stepper: one Lanczos iteration for many solves at once ----------
//
// Same recurrence, start vector, stop rule and arithmetic as run_lanczos,
// but alpha and beta stay on the device (kernels read them through
// pointers), the products of all active solves run as one fused launch, and
// a step ends with one copy of every solve's (alpha, beta) and one sync.

namespace {

// w -= alpha v + beta_prev vp with alpha = s[0].x and beta_prev = *bp
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) k_three_term_dev(void *pw, const void *pv, const void *pvp, uint64_t n,
                                                           const double2 *s, const double *bp) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const double alpha = s[0].x;
    const double beta = pvp ? *bp : 0.0;
    if constexpr (CPLX) {
        double2 w = static_cast<double2 *>(pw)[i];
        const double2 v = static_cast<const double2 *>(pv)[i];
        w.x -= alpha * v.x;
        w.y -= alpha * v.y;
        if (pvp) {
            const double2 u = static_cast<const double2 *>(pvp)[i];
            w.x -= beta * u.x;
            w.y -= beta * u.y;
        }
        static_cast<double2 *>(pw)[i] = w;
    } else {
        double w = static_cast<double *>(pw)[i];
        w -= alpha * static_cast<const double *>(pv)[i];
        if (pvp) w -= beta * static_cast<const double *>(pvp)[i];
        static_cast<double *>(pw)[i] = w;
    }
}

// scal[0] = alpha (from the reduced dot), scal[1] = sqrt(reduced norm^2)
__global__ void k_alpha_beta(const double2 *dot_a, const double2 *dot_b, double *scal) {
    scal[0] = dot_a[0].x;
    scal[1] = __dsqrt_rn(dot_b[0].x);   // correctly rounded, as std::sqrt on the host
}

__global__ void __launch_bounds__(kBlock) k_div_dev(double *dst, const double *src, uint64_t n, const double *s) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i] / *s;
}

}  // namespace

}  // namespace ls

struct ls_solver {
    const ls_operator *op = nullptr;
    bool cplx = false;
    uint64_t n = 0;
    uint32_t m = 0;
    double tol = 0.0;
    int reorth = 1;               // none, full CGS2, selective second pass
    void *V = nullptr;            // [m][n]
    void *w = nullptr;            // [n]
    double2 *partial = nullptr;   // [kDotBlocks][m]
    double2 *hs = nullptr;        // [m] reorthogonalisation coefficients
    void *aux = nullptr;          // norms and gate of the reorthogonalisation
    double2 *dots = nullptr;      // [2]: <v_k, w>, <w, w>
    double *scal = nullptr;       // [2]: alpha_k, beta_{k+1}
    double *bprev = nullptr;      // beta_k (device copy)
    double *host = nullptr;       // pinned [2]
    uint32_t *hflag = nullptr;    // pinned: the operator's error flag after a step
    std::vector<double> alpha, beta;
    uint32_t k = 0;
    double e0 = 0.0, resid = INFINITY, prev = 0.0;
    bool have_prev = false, done = false, converged = false;
    bool failed = false;          // a product met a lookup miss (LS_EINTERNAL)
};

namespace ls {

namespace {
std::mutex g_step_mu;
FusedState *g_fused = nullptr;

void free_solver(ls_solver *s) {
    if (!s) return;
    hipFree(s->V);
    hipFree(s->w);
    hipFree(s->partial);
    hipFree(s->hs);
    hipFree(s->aux);
    hipFree(s->dots);
    hipFree(s->scal);
    hipFree(s->bprev);
    if (s->host) hipHostFree(s->host);
    if (s->hflag) hipHostFree(s->hflag);
    delete s;
}

template <bool CPLX>
void enqueue_dot(ls_solver *s, const void *a, const void *b, double2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial<CPLX>, dim3(kDotBlocks), dim3(kBlock), 0, st, a, b, s->n, s->partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, s->partial, kDotBlocks, 1, out);
}

// everything of step k after the product
template <bool CPLX>
void enqueue_after_product(ls_solver *s, hipStream_t st) {
    using T = typename V<CPLX>::T;
    const uint64_t n = s->n;
    T *Vb = static_cast<T *>(s->V);
    T *w = static_cast<T *>(s->w);
    const uint32_t k = s->k;
    T *vk = Vb + static_cast<uint64_t>(k) * n;
    enqueue_dot<CPLX>(s, vk, w, s->dots, st);
    hipLaunchKernelGGL(k_three_term_dev<CPLX>, dim3(grid(n)), dim3(kBlock), 0, st, w, vk,
                       k > 0 ? Vb + static_cast<uint64_t>(k - 1) * n : nullptr, n, s->dots, s->bprev);
    const ReorthBufs rb = reorth_bufs(s->partial, s->hs, s->aux, static_cast<int>(s->m));
    enqueue_reorth<CPLX>(Vb, n, static_cast<int>(k) + 1, s->reorth, w, rb, s->dots + 1, st);
    hipLaunchKernelGGL(k_alpha_beta, dim3(1), dim3(1), 0, st, s->dots, s->dots + 1, s->scal);
    if (k + 1 < s->m) {
        const uint64_t nd = n * (CPLX ? 2 : 1);
        hipLaunchKernelGGL(k_div_dev, dim3(grid(nd)), dim3(kBlock), 0, st,
                           reinterpret_cast<double *>(Vb + static_cast<uint64_t>(k + 1) * n),
                           reinterpret_cast<const double *>(w), nd, s->scal + 1);
        LS_HIP_CHECK(hipMemcpyAsync(s->bprev, s->scal + 1, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    LS_HIP_CHECK(hipMemcpyAsync(s->host, s->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    enqueue_flag_read(s->op, s->hflag, st);
    LS_HIP_CHECK(hipGetLastError());
}

// host bookkeeping of step k, identical to run_lanczos
void finish_step(ls_solver *s) {
    const double a = s->host[0], bnext = s->host[1];
    s->alpha.push_back(a);
    s->e0 = tridiag_lowest(s->alpha, s->beta);
    s->resid = bnext * tridiag_last_component(s->alpha, s->beta, s->e0);
    const double scale = std::max(1.0, std::fabs(s->e0));
    if (s->tol > 0 && s->have_prev && std::fabs(s->e0 - s->prev) < s->tol * scale &&
        s->resid < std::sqrt(s->tol) * scale) {
        s->converged = true;
        s->done = true;
        return;
    }
    s->prev = s->e0;
    s->have_prev = true;
    s->k += 1;
    if (s->k >= s->m || bnext == 0.0) {
        s->done = true;
        return;
    }
    s->beta.push_back(bnext);
}

}  // namespace

uint64_t solver_footprint(const ls_operator *op, uint32_t max_iter) {
    const uint64_t n = op->basis->dim;
    const uint64_t m = std::min<uint64_t>(max_iter, n);
    const uint64_t es = op->is_complex ? 16 : 8;
    return (m + 1) * n * es + static_cast<uint64_t>(kDotBlocks) * std::max<uint64_t>(m, 1) * 16 + kAuxBytes + 4096;
}

ls_solver *solver_create(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t st) {
    ls_solver *s = new ls_solver();
    try {
        s->op = op;
        s->cplx = op->is_complex;
        s->n = op->basis->dim;
        s->m = static_cast<uint32_t>(std::min<uint64_t>(o->max_iter, s->n));
        s->tol = o->tol;
        s->reorth = static_cast<int>(o->reorth);
        const size_t es = s->cplx ? 16 : 8;
        if (hipMalloc(&s->V, static_cast<size_t>(s->m) * s->n * es) != hipSuccess)
            throw Error{LS_ENOMEM, "cannot allocate the Krylov vectors"};
        LS_HIP_CHECK(hipMalloc(&s->w, s->n * es));
        LS_HIP_CHECK(hipMalloc(&s->partial, static_cast<size_t>(kDotBlocks) * std::max<uint32_t>(s->m, 1) *
                                                sizeof(double2)));
        LS_HIP_CHECK(hipMalloc(&s->hs, std::max<uint32_t>(s->m, 1) * sizeof(double2)));
        LS_HIP_CHECK(hipMalloc(&s->aux, kAuxBytes));
        LS_HIP_CHECK(hipMalloc(&s->dots, 2 * sizeof(double2)));
        LS_HIP_CHECK(hipMalloc(&s->scal, 2 * sizeof(double)));
        LS_HIP_CHECK(hipMalloc(&s->bprev, sizeof(double)));
        LS_HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&s->host), 2 * sizeof(double)));
        LS_HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&s->hflag), sizeof(uint32_t)));
        *s->hflag = 0;
        // start vector, normalised exactly as run_lanczos does
        const uint64_t nd = s->n * (s->cplx ? 2 : 1);
        if (o->d_v0)
            LS_HIP_CHECK(hipMemcpyAsync(s->w, o->d_v0, s->n * es, hipMemcpyDeviceToDevice, st));
        else
            hipLaunchKernelGGL(k_fill_uniform, dim3(grid(nd)), dim3(kBlock), 0, st, static_cast<double *>(s->w), nd,
                               o->seed);
        if (s->cplx) enqueue_dot<true>(s, s->w, s->w, s->dots, st);
        else enqueue_dot<false>(s, s->w, s->w, s->dots, st);
        double2 r;
        LS_HIP_CHECK(hipMemcpyAsync(&r, s->dots, sizeof(double2), hipMemcpyDeviceToHost, st));
        LS_HIP_CHECK(hipStreamSynchronize(st));
        const double nrm0 = std::sqrt(r.x);
        if (!(nrm0 > 0.0)) throw Error{LS_EINVAL, "the start vector is zero"};
        hipLaunchKernelGGL(k_div, dim3(grid(nd)), dim3(kBlock), 0, st, static_cast<double *>(s->V),
                           static_cast<const double *>(s->w), nd, nrm0);
        LS_HIP_CHECK(hipGetLastError());
        LS_HIP_CHECK(hipStreamSynchronize(st));
    } catch (...) {
        free_solver(s);
        throw;
    }
    return s;
}

void solver_destroy(ls_solver *s) {
    hipDeviceSynchronize();
    free_solver(s);
}

void solver_step(ls_solver *const *ss, uint32_t n, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_step_mu);
    if (!g_fused) g_fused = fused_create();
    std::vector<ls_solver *> act;
    for (uint32_t i = 0; i < n; ++i)
        if (ss[i] && !ss[i]->done) act.push_back(ss[i]);
    if (act.empty()) return;
    // one fused launch for every active solve's product w = H v_k
    std::vector<const ls_operator *> ops;
    std::vector<const void *> xs;
    std::vector<void *> ys;
    for (ls_solver *s : act) {
        const size_t es = s->cplx ? 16 : 8;
        ops.push_back(s->op);
        xs.push_back(static_cast<const char *>(s->V) + static_cast<size_t>(s->k) * s->n * es);
        ys.push_back(s->w);
    }
    // a solve whose operator holds stored elements takes its stored product;
    // the others share one fused launch, or take the single launch when
    // alone (its tuned shape).  The row arithmetic, and so every result bit,
    // is the same in all three.
    std::vector<const ls_operator *> fops;
    std::vector<const void *> fxs;
    std::vector<void *> fys;
    for (size_t i = 0; i < ops.size(); ++i) {
        if (ops[i]->stored) {
            launch_matvec(ops[i], 1, xs[i], ys[i], st);
        } else {
            fops.push_back(ops[i]);
            fxs.push_back(xs[i]);
            fys.push_back(ys[i]);
        }
    }
    if (fops.size() == 1) launch_matvec(fops[0], 1, fxs[0], fys[0], st);
    else if (fops.size() > 1)
        fused_matvec(g_fused, static_cast<uint32_t>(fops.size()), fops.data(), fxs.data(), fys.data(), st);
    for (ls_solver *s : act) {
        if (s->cplx) enqueue_after_product<true>(s, st);
        else enqueue_after_product<false>(s, st);
    }
    LS_HIP_CHECK(hipStreamSynchronize(st));
    // a solve whose product met a lookup miss stops here (its step is not
    // taken); the others finish theirs
    uint32_t failed = 0;
    for (ls_solver *s : act) {
        if (*s->hflag) {
            *s->hflag = 0;
            s->failed = true;
            s->done = true;
            ++failed;
        } else {
            finish_step(s);
        }
    }
    if (failed)
        throw Error{LS_EINTERNAL, std::to_string(failed) + " of " + std::to_string(act.size()) +
                                      " solves met a neighbour whose representative lies in the sector but is "
                                      "missing from the basis; they are stopped (ls_solver_result reports them)"};
}

bool solver_failed(const ls_solver *s) { return s->failed; }

void solver_result(const ls_solver *s, double *e0, uint32_t *iters, double *resid, int *done, int *converged) {
    if (e0) *e0 = s->e0;
    if (iters) *iters = static_cast<uint32_t>(s->alpha.size());
    if (resid) *resid = s->resid;
    if (done) *done = s->done ? 1 : 0;
    if (converged) *converged = s->converged ? 1 : 0;
}

}  // namespace ls
