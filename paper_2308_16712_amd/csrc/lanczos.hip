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
// iteration for the last component of its eigenvector).  ls_lanczos runs
// one solve through the stepper below: alpha and beta stay on the device and
// a step ends with one synchronisation.

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

}  // namespace

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
    double host_rows[2] = {0.0, 0.0};
    uint32_t hflag_word = 0;
    double *host = host_rows;     // [2] alpha, beta read back after a step
    uint32_t *hflag = &hflag_word;   // the operator's error flag after a step
    ls::StreamSet used;           // streams of its steps
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
    s->used.drain();
    dev_free(s->V);
    dev_free(s->w);
    dev_free(s->partial);
    dev_free(s->hs);
    dev_free(s->aux);
    dev_free(s->dots);
    dev_free(s->scal);
    dev_free(s->bprev);
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
        s->used.add(st);
        try {
            s->V = dev_alloc(static_cast<size_t>(s->m) * s->n * es, st);
        } catch (const Error &) {
            throw Error{LS_ENOMEM, "cannot allocate the Krylov vectors"};
        }
        s->w = dev_alloc(s->n * es, st);
        s->partial = dev_alloc_n<double2>(static_cast<size_t>(kDotBlocks) * std::max<uint32_t>(s->m, 1), st);
        s->hs = dev_alloc_n<double2>(std::max<uint32_t>(s->m, 1), st);
        s->aux = dev_alloc(kAuxBytes, st);
        s->dots = dev_alloc_n<double2>(2, st);
        s->scal = dev_alloc_n<double>(2, st);
        s->bprev = dev_alloc_n<double>(1, st);
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

void solver_destroy(ls_solver *s) { free_solver(s); }

// ---- batched step: the work after the products of several solves, one
// launch per kernel for all of them ------------------------------------------
//
// A step of a single solve runs about thirty small kernels (dot products,
// the three-term update, two Gram-Schmidt passes in tiles of eight vectors,
// reductions, the normalisation); over many small solves those launches, not
// the GPU, set the step time.  Here each kernel runs once for all solves of
// the step: its flat grid is mapped onto (solve, block) pairs through prefix
// tables.  Every block computes exactly the partial sums the single kernels
// compute for the non-empty blocks of the fixed 2048-block dot grid (the
// same element sets, accumulation order and reduction tree), and the
// reductions read the missing partials as the zeros that the empty blocks
// of the single kernels write, so a solve gets the same bits alone or here.

namespace {

struct StepJob {
    const void *V;        // [m][n] Krylov vectors
    void *w;              // [n]
    uint64_t n;
    uint32_t k, m;        // step, Krylov dimension cap
    uint32_t nb;          // non-empty blocks of the dot grid: min(2048, ceil(n / 256))
    uint32_t mode;        // reorthogonalisation: none, full, selective
    uint32_t last;        // k + 1 == m: no next vector is formed
    uint32_t pad_;
    double2 *partial;     // [kDotBlocks][m]
    double2 *hs;          // [m]
    double2 *npart;       // [2][kDotBlocks] block parts of ||w||^2 before / after a pass
    double2 *nrm;         // [4]
    int *gate;            // second Gram-Schmidt pass needed
    double2 *dots;        // [2]: <v_k, w>, ||w||^2
    double *scal;         // [2]: alpha_k, beta_{k+1}
    double *bprev;        // beta_k
    uint32_t *err;        // the operator's lookup-miss flag
    double *row;          // [4] device staging row: alpha, beta, flag (read back in one copy)
};

// One reduction of 2048 virtual block partials into one output (the loop
// and tree of k_reduce_partials); partials at or beyond nb are zeros.
struct RedTask {
    const double2 *src;   // partial b of output j at src[b * stride + j]
    uint32_t stride, nb, nout, pad_;
    double2 *dst;         // dst[j], j < nout
};

// Index of the segment holding flat block index x: off[0] = 0 <= ... <= off[count].
__device__ __forceinline__ uint32_t segment_of(const uint32_t *off, uint32_t count, uint32_t x) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kBlock) kb_reduce(const RedTask *tasks, const uint32_t *off, uint32_t count) {
    __shared__ double sh[kBlock];
    const uint32_t t = segment_of(off, count, blockIdx.x);
    const RedTask T = tasks[t];
    const uint32_t j = blockIdx.x - off[t];
    double re = 0.0, im = 0.0;
    for (uint32_t b = threadIdx.x; b < static_cast<uint32_t>(kDotBlocks); b += kBlock) {
        const double2 v = b < T.nb ? T.src[static_cast<size_t>(b) * T.stride + j] : make_double2(0.0, 0.0);
        re += v.x;
        im += v.y;
    }
    re = block_reduce(re, sh);
    im = block_reduce(im, sh);
    if (threadIdx.x == 0) T.dst[j] = make_double2(re, im);
}

// partial[b] = the block's part of <a, b> (k_dot_partial) with a = v_k, b = w
// (which = 0) or a = b = w (which = 1, written to partial too)
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) kb_dot(const StepJob *jobs, const uint32_t *off, uint32_t count, int which) {
    using T = typename V<CPLX>::T;
    __shared__ double sh[kBlock];
    const uint32_t s = segment_of(off, count, blockIdx.x);
    const StepJob &J = jobs[s];
    const uint32_t b = blockIdx.x - off[s];
    const T *pa = which == 0 ? static_cast<const T *>(J.V) + static_cast<uint64_t>(J.k) * J.n
                             : static_cast<const T *>(J.w);
    const T *pb = static_cast<const T *>(J.w);
    double re = 0.0, im = 0.0;
    const uint64_t stride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (uint64_t i = static_cast<uint64_t>(b) * kBlock + threadIdx.x; i < J.n; i += stride) {
        if constexpr (CPLX) {
            const double2 x = pa[i], y = pb[i];
            re = fma(x.x, y.x, fma(x.y, y.y, re));
            im = fma(x.x, y.y, fma(-x.y, y.x, im));
        } else {
            re = fma(pa[i], pb[i], re);
        }
    }
    re = block_reduce(re, sh);
    if constexpr (CPLX) im = block_reduce(im, sh);
    if (threadIdx.x == 0) J.partial[b] = make_double2(re, im);
}

// w -= alpha v_k + beta_k v_{k-1}, elementwise (k_three_term_dev)
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) kb_three_term(const StepJob *jobs, const uint32_t *off, uint32_t count) {
    using T = typename V<CPLX>::T;
    const uint32_t s = segment_of(off, count, blockIdx.x);
    const StepJob &J = jobs[s];
    const uint64_t i = static_cast<uint64_t>(blockIdx.x - off[s]) * kBlock + threadIdx.x;
    if (i >= J.n) return;
    const T *Vb = static_cast<const T *>(J.V);
    const T *pv = Vb + static_cast<uint64_t>(J.k) * J.n;
    const T *pvp = J.k > 0 ? Vb + static_cast<uint64_t>(J.k - 1) * J.n : nullptr;
    const double alpha = J.dots[0].x;
    const double beta = pvp ? *J.bprev : 0.0;
    T *pw = static_cast<T *>(J.w);
    if constexpr (CPLX) {
        double2 w = pw[i];
        const double2 v = pv[i];
        w.x -= alpha * v.x;
        w.y -= alpha * v.y;
        if (pvp) {
            const double2 u = pvp[i];
            w.x -= beta * u.x;
            w.y -= beta * u.y;
        }
        pw[i] = w;
    } else {
        double w = pw[i];
        w -= alpha * pv[i];
        if (pvp) w -= beta * pvp[i];
        pw[i] = w;
    }
}

// Gram-Schmidt pass `pass` (k_multidot_partial for every tile of eight
// vectors of V_0 .. V_k, in order); the selective mode's second pass runs
// only when the gate is set, and its first pass also records ||w||^2.
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) kb_multidot(const StepJob *jobs, const uint32_t *off, uint32_t count,
                                                      int pass) {
    __shared__ double sh[kBlock];
    const uint32_t s = segment_of(off, count, blockIdx.x);
    const StepJob &J = jobs[s];
    const bool sel = J.mode == kReorthSelective;
    if (sel && pass == 1 && *J.gate == 0) return;
    const uint32_t b = blockIdx.x - off[s];
    const int nv = static_cast<int>(J.k) + 1;
    const uint64_t n = J.n;
    const uint64_t gstride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (int j0 = 0; j0 < nv; j0 += kTile) {
        const int tile = min(kTile, nv - j0);
        const bool wn = sel && pass == 0 && j0 == 0;
        double re[kTile], im[kTile];
        double nre = 0.0;
#pragma unroll
        for (int q = 0; q < kTile; ++q) re[q] = im[q] = 0.0;
        for (uint64_t i = static_cast<uint64_t>(b) * kBlock + threadIdx.x; i < n; i += gstride) {
            if constexpr (CPLX) {
                const double2 w = static_cast<const double2 *>(J.w)[i];
                if (wn) nre = fma(w.x, w.x, fma(w.y, w.y, nre));
                const double2 *Vb = static_cast<const double2 *>(J.V);
#pragma unroll
                for (int q = 0; q < kTile; ++q) {
                    if (q < tile) {
                        const double2 v = Vb[static_cast<uint64_t>(j0 + q) * n + i];
                        re[q] = fma(v.x, w.x, fma(v.y, w.y, re[q]));
                        im[q] = fma(v.x, w.y, fma(-v.y, w.x, im[q]));
                    }
                }
            } else {
                const double w = static_cast<const double *>(J.w)[i];
                if (wn) nre = fma(w, w, nre);
                const double *Vb = static_cast<const double *>(J.V);
#pragma unroll
                for (int q = 0; q < kTile; ++q)
                    if (q < tile) re[q] = fma(Vb[static_cast<uint64_t>(j0 + q) * n + i], w, re[q]);
            }
        }
        for (int q = 0; q < tile; ++q) {
            const double r = block_reduce(re[q], sh);
            double m = 0.0;
            if constexpr (CPLX) m = block_reduce(im[q], sh);
            if (threadIdx.x == 0) J.partial[static_cast<size_t>(b) * J.m + j0 + q] = make_double2(r, m);
        }
        if (wn) {
            const double r = block_reduce(nre, sh);
            if (threadIdx.x == 0) J.npart[b] = make_double2(r, 0.0);
        }
    }
}

// w -= sum_j V_j h_j with the block part of the new ||w||^2 (k_gemv_sub)
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) kb_gemv_sub(const StepJob *jobs, const uint32_t *off, uint32_t count,
                                                      int pass) {
    __shared__ double sh[kBlock];
    const uint32_t s = segment_of(off, count, blockIdx.x);
    const StepJob &J = jobs[s];
    const bool sel = J.mode == kReorthSelective;
    if (sel && pass == 1 && *J.gate == 0) return;
    const uint32_t b = blockIdx.x - off[s];
    const int nv = static_cast<int>(J.k) + 1;
    const uint64_t n = J.n;
    const double2 *h = J.hs;
    double nre = 0.0;
    const uint64_t gstride = static_cast<uint64_t>(kDotBlocks) * kBlock;
    for (uint64_t i = static_cast<uint64_t>(b) * kBlock + threadIdx.x; i < n; i += gstride) {
        if constexpr (CPLX) {
            const double2 *Vb = static_cast<const double2 *>(J.V);
            double2 w = static_cast<double2 *>(J.w)[i];
            double sre = 0.0, sim = 0.0;
            for (int j = 0; j < nv; ++j) {
                const double2 v = Vb[static_cast<uint64_t>(j) * n + i];
                const double2 c = h[j];
                sre = fma(v.x, c.x, fma(-v.y, c.y, sre));
                sim = fma(v.x, c.y, fma(v.y, c.x, sim));
            }
            w.x -= sre;
            w.y -= sim;
            static_cast<double2 *>(J.w)[i] = w;
            nre = fma(w.x, w.x, fma(w.y, w.y, nre));
        } else {
            const double *Vb = static_cast<const double *>(J.V);
            double acc = 0.0;
            for (int j = 0; j < nv; ++j) acc = fma(Vb[static_cast<uint64_t>(j) * n + i], h[j].x, acc);
            const double w = static_cast<double *>(J.w)[i] - acc;
            static_cast<double *>(J.w)[i] = w;
            nre = fma(w, w, nre);
        }
    }
    if (sel || pass == 1) {
        const double r = block_reduce(nre, sh);
        if (threadIdx.x == 0) J.npart[kDotBlocks + b] = make_double2(r, 0.0);
    }
}

// per solve (one thread each): the selective test after the first pass
// (k_reorth_decide), or the norm of the pass that ran (k_reorth_pick)
__global__ void kb_decide(const StepJob *jobs, uint32_t count, int stage) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const StepJob &J = jobs[s];
    if (J.mode != kReorthSelective) return;
    if (stage == 0) {
        *J.gate = J.nrm[1].x < 0.5 * J.nrm[0].x ? 1 : 0;
        J.dots[1] = J.nrm[1];
    } else if (*J.gate) {
        J.dots[1] = J.nrm[2];
    }
}

// per solve: alpha, beta (k_alpha_beta), beta_k for the next step, and the
// staging row read back by the host (alpha, beta, lookup-miss flag; the
// flags are cleared before the next step's products, so solves sharing an
// operator all see its flag)
__global__ void kb_alpha_beta(const StepJob *jobs, uint32_t count) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const StepJob &J = jobs[s];
    J.scal[0] = J.dots[0].x;
    J.scal[1] = __dsqrt_rn(J.dots[1].x);
    J.row[0] = J.scal[0];
    J.row[1] = J.scal[1];
    J.row[2] = static_cast<double>(*J.err);
}

// Clears up to 32 operators' lookup-miss flags (a fill kernel, not a memset).
struct FlagList {
    uint32_t *p[32];
    uint32_t n;
};
__global__ void k_clear_flags(FlagList L) {
    if (threadIdx.x < L.n) *L.p[threadIdx.x] = 0u;
}

// V_{k+1} = w / beta_{k+1} elementwise over doubles (k_div_dev), and beta_k
// for the next step
template <bool CPLX>
__global__ void __launch_bounds__(kBlock) kb_div(const StepJob *jobs, const uint32_t *off, uint32_t count) {
    const uint32_t s = segment_of(off, count, blockIdx.x);
    const StepJob &J = jobs[s];
    if (J.last) return;
    const uint64_t nd = J.n * (CPLX ? 2 : 1);
    const uint64_t i = static_cast<uint64_t>(blockIdx.x - off[s]) * kBlock + threadIdx.x;
    if (i == 0) *J.bprev = J.scal[1];
    if (i >= nd) return;
    double *dst = static_cast<double *>(const_cast<void *>(J.V)) + (static_cast<uint64_t>(J.k) + 1) * nd;
    dst[i] = static_cast<const double *>(J.w)[i] / J.scal[1];
}

// Device tables of a batched step, grown by doubling and reused.
struct StepTables {
    StepJob *jobs = nullptr;
    RedTask *tasks = nullptr;
    uint32_t *offs = nullptr;     // prefix tables, packed
    double *staging = nullptr;    // [count][4] device side of the read-back
    size_t cap_jobs = 0, cap_tasks = 0, cap_offs = 0, cap_staging = 0;
};
StepTables g_tables;

template <typename X>
void grow(X **p, size_t *cap, size_t need) {
    if (need <= *cap) return;
    const size_t c = std::max<size_t>(need, *cap * 2 + 16);
    if (*p) LS_HIP_CHECK(hipFree(*p));
    *p = nullptr;
    LS_HIP_CHECK(hipMalloc(p, c * sizeof(X)));
    *cap = c;
}

}  // namespace

// The after-product work of step k for every solve in `act`, batched: all
// of one element type, and either all reorthogonalising (full or selective,
// mixed) or none.  Each solve's (alpha, beta, flag) row lands in host_rows
// ([act][4], pinned) on `st`; the host tables it uploads go to `keep`.
template <bool CPLX>
void batched_after_products(const std::vector<ls_solver *> &act, hipStream_t st, double *host_rows, HostKeep &keep) {
    const uint32_t S = static_cast<uint32_t>(act.size());
    StepTables &G = g_tables;   // sized by the caller for the whole step
    std::vector<StepJob> jobs(S);
    std::vector<uint32_t> off_dot(S + 1, 0), off_el(S + 1, 0), off_div(S + 1, 0), o_one(S + 1), o_h(S + 1, 0);
    bool none = false;
    for (uint32_t i = 0; i < S; ++i) {
        ls_solver *sv = act[i];
        StepJob &J = jobs[i];
        J.V = sv->V;
        J.w = sv->w;
        J.n = sv->n;
        J.k = sv->k;
        J.m = sv->m;
        J.nb = static_cast<uint32_t>(std::min<uint64_t>(kDotBlocks, (sv->n + kBlock - 1) / kBlock));
        J.mode = static_cast<uint32_t>(sv->reorth);
        J.last = sv->k + 1 >= sv->m ? 1u : 0u;
        const ReorthBufs rb = reorth_bufs(sv->partial, sv->hs, sv->aux, static_cast<int>(sv->m));
        J.partial = rb.partial;
        J.hs = rb.hs;
        J.npart = rb.npart;
        J.nrm = rb.nrm;
        J.gate = rb.gate;
        J.dots = sv->dots;
        J.scal = sv->scal;
        J.bprev = sv->bprev;
        J.err = sv->op->d_err;
        J.row = G.staging + 4 * static_cast<size_t>(i);
        none = J.mode == kReorthNone;
        off_dot[i + 1] = off_dot[i] + J.nb;
        off_el[i + 1] = off_el[i] + static_cast<uint32_t>((sv->n + kBlock - 1) / kBlock);
        const uint64_t nd = sv->n * (CPLX ? 2 : 1);
        off_div[i + 1] = off_div[i] + static_cast<uint32_t>((nd + kBlock - 1) / kBlock);
        o_one[i] = i;
        o_h[i + 1] = o_h[i] + J.k + 1;
    }
    o_one[S] = S;
    // reduction tasks: alpha, h, ||w||^2 before / after the first pass, the
    // final ||w||^2 (after the second pass, or without reorthogonalisation)
    std::vector<RedTask> tasks;
    tasks.reserve(5 * static_cast<size_t>(S));
    for (const StepJob &J : jobs) tasks.push_back(RedTask{J.partial, 1, J.nb, 1, 0, J.dots});
    for (const StepJob &J : jobs) tasks.push_back(RedTask{J.partial, J.m, J.nb, J.k + 1, 0, J.hs});
    for (const StepJob &J : jobs) tasks.push_back(RedTask{J.npart, 1, J.nb, 1, 0, J.nrm});
    for (const StepJob &J : jobs)
        tasks.push_back(RedTask{J.npart + kDotBlocks, 1, J.nb, 1, 0, J.mode == kReorthSelective ? J.nrm + 1 : J.nrm + 3});
    for (const StepJob &J : jobs)
        tasks.push_back(none ? RedTask{J.partial, 1, J.nb, 1, 0, J.dots + 1}
                             : RedTask{J.npart + kDotBlocks, 1, J.nb, 1, 0,
                                       J.mode == kReorthSelective ? J.nrm + 2 : J.dots + 1});
    std::vector<uint32_t> offs;
    for (auto *L : {&off_dot, &off_el, &off_div, &o_one, &o_h}) offs.insert(offs.end(), L->begin(), L->end());
    // uploaded from copies that live until the caller's synchronisation
    LS_HIP_CHECK(hipMemcpyAsync(G.jobs, keep_copy(keep, jobs.data(), jobs.size()), S * sizeof(StepJob),
                                hipMemcpyHostToDevice, st));
    LS_HIP_CHECK(hipMemcpyAsync(G.tasks, keep_copy(keep, tasks.data(), tasks.size()), tasks.size() * sizeof(RedTask),
                                hipMemcpyHostToDevice, st));
    LS_HIP_CHECK(hipMemcpyAsync(G.offs, keep_copy(keep, offs.data(), offs.size()), offs.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, st));
    const uint32_t *d_dot = G.offs, *d_el = d_dot + (S + 1), *d_div = d_el + (S + 1), *d_one = d_div + (S + 1),
                   *d_h = d_one + (S + 1);
    const RedTask *T_alpha = G.tasks, *T_h = T_alpha + S, *T_before = T_h + S, *T_after = T_before + S,
                  *T_final = T_after + S;
    const dim3 blk(kBlock);
    const uint32_t per = 64;   // solves per block of the per-solve kernels
    const dim3 gs((S + per - 1) / per);
    // alpha = <v_k, w>
    hipLaunchKernelGGL(kb_dot<CPLX>, dim3(off_dot[S]), blk, 0, st, G.jobs, d_dot, S, 0);
    hipLaunchKernelGGL(kb_reduce, dim3(S), blk, 0, st, T_alpha, d_one, S);
    // w -= alpha v_k + beta_k v_{k-1}
    hipLaunchKernelGGL(kb_three_term<CPLX>, dim3(off_el[S]), blk, 0, st, G.jobs, d_el, S);
    if (none) {
        // ||w||^2 directly
        hipLaunchKernelGGL(kb_dot<CPLX>, dim3(off_dot[S]), blk, 0, st, G.jobs, d_dot, S, 1);
    } else {
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(kb_multidot<CPLX>, dim3(off_dot[S]), blk, 0, st, G.jobs, d_dot, S, pass);
            hipLaunchKernelGGL(kb_reduce, dim3(o_h[S]), blk, 0, st, T_h, d_h, S);
            hipLaunchKernelGGL(kb_gemv_sub<CPLX>, dim3(off_dot[S]), blk, 0, st, G.jobs, d_dot, S, pass);
            if (pass == 0) {
                hipLaunchKernelGGL(kb_reduce, dim3(S), blk, 0, st, T_before, d_one, S);
                hipLaunchKernelGGL(kb_reduce, dim3(S), blk, 0, st, T_after, d_one, S);
                hipLaunchKernelGGL(kb_decide, gs, dim3(per), 0, st, G.jobs, S, 0);
            }
        }
    }
    hipLaunchKernelGGL(kb_reduce, dim3(S), blk, 0, st, T_final, d_one, S);
    if (!none) hipLaunchKernelGGL(kb_decide, gs, dim3(per), 0, st, G.jobs, S, 1);
    hipLaunchKernelGGL(kb_alpha_beta, gs, dim3(per), 0, st, G.jobs, S);
    hipLaunchKernelGGL(kb_div<CPLX>, dim3(off_div[S]), blk, 0, st, G.jobs, d_div, S);
    LS_HIP_CHECK(hipGetLastError());
    LS_HIP_CHECK(hipMemcpyAsync(host_rows, G.staging, S * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
}

namespace {

// Pinned read-back of a chunk of steps: [steps][solves][4] doubles (alpha,
// beta, flag) and [steps] flag words of a single solve.
struct StepRows {
    double *rows = nullptr;
    uint32_t *flags = nullptr;
    size_t cap_rows = 0, cap_flags = 0;
};
StepRows g_rows;

void ensure_rows(size_t n_rows, size_t n_flags) {
    if (g_rows.cap_rows < n_rows) {
        if (g_rows.rows) LS_HIP_CHECK(hipHostFree(g_rows.rows));
        g_rows.rows = nullptr;
        g_rows.cap_rows = 0;
        const size_t c = std::max<size_t>(n_rows, 2 * g_rows.cap_rows + 256);
        LS_HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&g_rows.rows), c * 4 * sizeof(double)));
        g_rows.cap_rows = c;
    }
    if (g_rows.cap_flags < n_flags) {
        if (g_rows.flags) LS_HIP_CHECK(hipHostFree(g_rows.flags));
        g_rows.flags = nullptr;
        g_rows.cap_flags = 0;
        const size_t c = std::max<size_t>(n_flags, 256);
        LS_HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&g_rows.flags), c * sizeof(uint32_t)));
        g_rows.cap_flags = c;
    }
}

}  // namespace

// Up to `steps` iterations of every listed solve that is not done, enqueued
// back to back with one synchronisation at the end.  Every kernel of a step
// reads alpha and beta on the device, so the steps need nothing from the
// host in between; each step's (alpha, beta, flag) rows land in pinned
// memory, and the host bookkeeping then replays the steps in order exactly
// as after single steps, stopping each solve where single steps would have
// stopped.  Steps enqueued past a solve's stop (convergence or breakdown
// inside the chunk) only write Krylov vectors and device scalars that the
// finished solve never reads.
void solver_step(ls_solver *const *ss, uint32_t n, uint32_t steps, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_step_mu);
    if (!g_fused) g_fused = fused_create();
    std::vector<ls_solver *> act;
    for (uint32_t i = 0; i < n; ++i)
        if (ss[i] && !ss[i]->done) act.push_back(ss[i]);
    if (act.empty() || steps == 0) return;
    uint32_t c = steps;
    for (ls_solver *s : act) {
        s->used.add(st);
        touch(s->op, st);
        c = std::min(c, s->m - s->k);   // k < m while a solve is not done
    }
    const size_t A = act.size();
    // the batched after-product kernels (one launch per kernel whatever the
    // Krylov dimension) also serve a lone small solve, whose step is bound by
    // launches (4x6 torus 0.38 -> 0.36 ms per step, 24-site ring 0.29 -> 0.26
    // ms); a large lone solve keeps the single kernels (32-site ring: 3.69 ms
    // against 4.10 ms batched).  Both give the same bits.
    const bool batched = A >= 2 || act[0]->n < (1ull << 21);
    std::vector<uint32_t> k0(A);
    for (size_t a = 0; a < A; ++a) k0[a] = act[a]->k;
    // operators' lookup-miss flags (cleared before each batched step's products)
    std::vector<uint32_t *> flags;
    for (ls_solver *s : act)
        if (std::find(flags.begin(), flags.end(), s->op->d_err) == flags.end()) flags.push_back(s->op->d_err);
    ensure_rows(A * c, c);
    // the work after the products: per solve for a single solve, else
    // batched by element type and reorthogonalisation (identical numbers)
    std::vector<ls_solver *> groups[4];   // (complex, without reorthogonalisation)
    std::vector<size_t> row_of(A, 0);
    if (batched) {
        StepTables &G = g_tables;
        grow(&G.jobs, &G.cap_jobs, A);
        grow(&G.staging, &G.cap_staging, 4 * A);
        grow(&G.tasks, &G.cap_tasks, 5 * A);
        grow(&G.offs, &G.cap_offs, 5 * (A + 1));
        std::vector<size_t> where[4];
        for (size_t a = 0; a < A; ++a) {
            const int g = (act[a]->cplx ? 2 : 0) + (act[a]->reorth == kReorthNone ? 1 : 0);
            groups[g].push_back(act[a]);
            where[g].push_back(a);
        }
        size_t r = 0;
        for (int g = 0; g < 4; ++g) {
            for (size_t q = 0; q < groups[g].size(); ++q) row_of[where[g][q]] = r + q;
            r += groups[g].size();
        }
    }
    double *const own_host = act[0]->host;
    uint32_t *const own_flag = act[0]->hflag;
    auto restore = [&]() {
        for (size_t a = 0; a < A; ++a) act[a]->k = k0[a];
        act[0]->host = own_host;
        act[0]->hflag = own_flag;
    };
    HostKeep keep;   // host sources of this chunk's uploads
    try {
        for (uint32_t i = 0; i < c; ++i) {
            for (size_t a = 0; a < A; ++a) act[a]->k = k0[a] + i;
            if (batched)
                for (size_t f = 0; f < flags.size(); f += 32) {
                    FlagList L{};
                    L.n = static_cast<uint32_t>(std::min<size_t>(32, flags.size() - f));
                    for (uint32_t q = 0; q < L.n; ++q) L.p[q] = flags[f + q];
                    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(32), 0, st, L);
                }
            // products w = H v_k: a solve whose operator holds stored elements
            // takes its stored product, a small sector its own row-group
            // launch; the others share one fused launch, or take the single
            // launch when alone.  Every form sums a row in term order, so
            // every result bit is the same in all of them.
            std::vector<const ls_operator *> fops;
            std::vector<const void *> fxs;
            std::vector<void *> fys;
            for (ls_solver *s : act) {
                const size_t es = s->cplx ? 16 : 8;
                const void *x = static_cast<const char *>(s->V) + static_cast<size_t>(s->k) * s->n * es;
                if (s->op->stored || grouped_product(s->op)) {
                    launch_matvec(s->op, 1, x, s->w, st);
                } else {
                    fops.push_back(s->op);
                    fxs.push_back(x);
                    fys.push_back(s->w);
                }
            }
            if (fops.size() == 1) launch_matvec(fops[0], 1, fxs[0], fys[0], st);
            else if (fops.size() > 1)
                fused_matvec(g_fused, static_cast<uint32_t>(fops.size()), fops.data(), fxs.data(), fys.data(), st,
                             &keep);
            if (!batched) {
                ls_solver *s = act[0];
                s->host = g_rows.rows + 4 * static_cast<size_t>(i);
                s->hflag = g_rows.flags + i;
                if (s->cplx) enqueue_after_product<true>(s, st);
                else enqueue_after_product<false>(s, st);
            } else {
                double *rows = g_rows.rows + 4 * A * static_cast<size_t>(i);
                size_t r = 0;
                for (int g = 0; g < 4; ++g) {
                    if (groups[g].empty()) continue;
                    if (g >= 2) batched_after_products<true>(groups[g], st, rows + 4 * r, keep);
                    else batched_after_products<false>(groups[g], st, rows + 4 * r, keep);
                    r += groups[g].size();
                }
            }
        }
        LS_HIP_CHECK(hipStreamSynchronize(st));
    } catch (...) {
        hipStreamSynchronize(st);   // the enqueued copies still read `keep`
        restore();
        throw;
    }
    restore();
    // replay: a solve whose product met a lookup miss stops at that step
    // (the step is not taken); the others finish theirs
    uint32_t failed = 0;
    double row2[2];
    for (uint32_t i = 0; i < c; ++i) {
        for (size_t a = 0; a < A; ++a) {
            ls_solver *s = act[a];
            if (s->done) continue;
            bool flag;
            double *saved = s->host;
            if (batched) {
                const double *row = g_rows.rows + 4 * (A * static_cast<size_t>(i) + row_of[a]);
                row2[0] = row[0];
                row2[1] = row[1];
                s->host = row2;
                flag = row[2] != 0.0;
            } else {
                s->host = g_rows.rows + 4 * static_cast<size_t>(i);
                flag = g_rows.flags[i] != 0;
            }
            if (flag) {
                s->failed = true;
                s->done = true;
                ++failed;
            } else {
                finish_step(s);
            }
            s->host = saved;
        }
    }
    if (failed)
        throw Error{LS_EINTERNAL, std::to_string(failed) + " of " + std::to_string(A) +
                                      " solves met a neighbour whose representative lies in the sector but is "
                                      "missing from the basis; they are stopped (ls_solver_result reports them)"};
}

bool solver_failed(const ls_solver *s) { return s->failed; }

// ls_lanczos: one solve driven by the stepper kernels (alpha and beta stay on
// the device), run in chunks of steps with one synchronisation per chunk.
// With a tolerance, sectors of up to 2^20 states run chunks of 8 steps (there
// a synchronisation costs about as much as a step; at most 7 steps run past
// convergence) and larger ones single steps; without a tolerance every step
// up to max_iter is needed and chunks hold 32 steps.  The arithmetic is that
// of single steps, kernel for kernel, so the results are those of
// ls_solver_step.
ls_status run_lanczos(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t st, double *e0_out,
                      uint32_t *iters_out, double *resid_out) {
    ls_solver *s = solver_create(op, o, st);
    const uint32_t chunk = o->tol > 0 ? (s->n <= (1u << 20) ? 8u : 1u) : 32u;
    try {
        while (!s->done) solver_step(&s, 1, chunk, st);
    } catch (...) {
        hipStreamSynchronize(st);
        free_solver(s);
        throw;
    }
    if (o->alpha)
        for (size_t k = 0; k < s->alpha.size(); ++k) o->alpha[k] = s->alpha[k];
    if (o->beta)
        for (size_t k = 0; k < s->beta.size(); ++k) o->beta[k] = s->beta[k];
    if (e0_out) *e0_out = s->e0;
    if (iters_out) *iters_out = static_cast<uint32_t>(s->alpha.size());
    if (resid_out) *resid_out = s->resid;
    const bool conv = s->converged;
    LS_HIP_CHECK(hipStreamSynchronize(st));
    free_solver(s);
    return (o->tol > 0 && !conv) ? LS_WNOTCONV : LS_OK;
}

void solver_result(const ls_solver *s, double *e0, uint32_t *iters, double *resid, int *done, int *converged) {
    if (e0) *e0 = s->e0;
    if (iters) *iters = static_cast<uint32_t>(s->alpha.size());
    if (resid) *resid = s->resid;
    if (done) *done = s->done ? 1 : 0;
    if (converged) *converged = s->converged ? 1 : 0;
}

}  // namespace ls
