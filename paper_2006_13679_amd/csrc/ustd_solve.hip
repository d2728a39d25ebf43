// ustd_solve.hip -- the pivot-column solve of the UST estimator of diag(L^+) on gfx950:
// L x = e_u - (1/n) 1 with x orthogonal to 1, which is column u of L^+ (Section "Overview",
// step 1; Algorithm 1, solver accuracy eta).  The paper solves it with conjugate gradients
// and the diagonal (Jacobi) preconditioner (Appendix "UST Generation, Pivot Selection, and
// the Linear System").
//
// Here CG runs with reliable updates: the solution x is accumulated in FP64, while the
// iteration itself runs on vectors of type T, FP64 or (mixed mode) FP32: the correction xs
// since the last update, the iterated residual rs, z = rs / diag, the direction p and q = L p.
// A reliable update folds xs into x and replaces rs by the true residual b - L x computed in
// FP64, keeping the direction p, so the Krylov space is not thrown away.  It is taken when
// |rs| has dropped by a factor delta since the largest residual after the previous update,
// when |rs| reaches the target, or at the iteration cap; the solve ends at an update whose
// true residual meets the target.  Dot products are accumulated in FP64 in a fixed order.
//
// Two engines: the whole solve in one workgroup (small graphs; many graphs of a batch side by
// side, one workgroup each), with no host round trip; or eight kernels per iteration whose
// scalars stay on the device, enqueued by the host in growing chunks ahead of a `done` flag that
// turns later launches into no-ops.
#include "ustd_kernels.hpp"

#include <algorithm>

namespace ustd {

constexpr int kSmallThreads = 1024;

// y = L p over all rows, degree-balanced: rows of degree <= heavy_thresh by groups of G lanes,
// heavier rows (listed in ascending order) by the whole block.  emit(v, (L p)_v) is called once
// per row from one thread.  Fixed grid and fixed per-row reduction trees: deterministic.
// Block blk of nblk takes every nblk-th heavy row and row tile (a whole grid: blockIdx.x of
// gridDim.x; a workgroup that solves a graph alone: 0 of 1).  BS = block size.
template <typename T, int G, int BS = 256, typename Emit>
__device__ __forceinline__ void lap_apply_rows(const RowMap &m, const T *__restrict__ p, Emit emit, int blk,
                                               int nblk) {
    __shared__ T shr[BS / kWave];
    const int nh = *m.nheavy;
    const double *__restrict__ w = m.w;  // uniform: weighted Laplacian when set
    for (int h = blk; h < nh; h += nblk) {
        const int v = m.heavy[h];
        const int lo = m.rp[v], hi = m.rp[v + 1];
        T acc = (T)0;
        if (w)
            for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) acc += (T)w[e] * p[m.col[e]];
        else
            for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) acc += p[m.col[e]];
        acc = block_sum_t<T>(acc, shr);
        if (threadIdx.x == 0) emit(v, (w ? (T)m.wdeg[v] : (T)(hi - lo)) * p[v] - acc);
    }
    constexpr int rows_per_tile = BS / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int tile = blk; tile * rows_per_tile < m.n; tile += nblk) {
        const int v = tile * rows_per_tile + g;
        const bool ok = v < m.n;
        const int lo = ok ? m.rp[v] : 0, hi = ok ? m.rp[v + 1] : 0;
        const bool light = ok && (hi - lo <= m.heavy_thresh);
        T acc = (T)0;
        if (light) {
            if (w)
                for (int e = lo + l; e < hi; e += G) acc += (T)w[e] * p[m.col[e]];
            else
                for (int e = lo + l; e < hi; e += G) acc += p[m.col[e]];
        }
#pragma unroll
        for (int dd = G / 2; dd > 0; dd >>= 1) acc += __shfl_xor(acc, dd, G);
        if (light && l == 0) emit(v, (w ? (T)m.wdeg[v] : (T)(hi - lo)) * p[v] - acc);
    }
}

// Jacobi diagonal: the degree, or the conductance sum of a weighted Laplacian's row
template <typename T>
__device__ __forceinline__ T jacobi_diag(const SolveArgs<T> &a, int v) {
    return a.wdeg ? (T)a.wdeg[v] : (T)(a.rp[v + 1] - a.rp[v]);
}

// right-hand side e_u - 1/n
__device__ __forceinline__ double rhs_of(int v, int u, double inv_n) { return (v == u ? 1.0 : 0.0) - inv_n; }

// Sum of per-block partials part[i * stride], i < nparts, in index order by one block.
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nparts, int stride, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[(long long)i * stride];
    return block_sum(v, sh);
}

// partial regions: p.q | (z.r, r.r) of the update | (z.r, |b - L x|^2) of a reliable update
__device__ __forceinline__ double *part_pq(double *part) { return part; }
__device__ __forceinline__ double *part_upd(double *part) { return part + kMaxSolveGrid; }
__device__ __forceinline__ double *part_rel(double *part) { return part + 3 * kMaxSolveGrid; }

// ---------------------------------------------------------------------------------------
// multi-kernel solve (large graphs): eight kernels per iteration, whose scalars stay on the
// device; once `done` is set every later launch of the solve returns at once.
// ---------------------------------------------------------------------------------------
// x = 0, xs = 0, rs = b, z = p = rs / diag; partials of z.r, r.r and b.b (3 per block)
template <typename T>
__global__ __launch_bounds__(256) void solve_start_kernel(SolveArgs<T> a) {
    __shared__ double sh[4];
    const double inv_n = 1.0 / (double)a.n;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        const double b = rhs_of(v, a.u, inv_n);
        const T rv = (T)b;
        const T zv = rv / jacobi_diag(a, v);
        a.x[v] = 0.0;
        a.xs[v] = (T)0;
        a.rs[v] = rv;
        a.z[v] = zv;
        a.p[v] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
        bb += b * b;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        double *pr = part_rel(a.part) + 3 * blockIdx.x;
        pr[0] = rz;
        pr[1] = rr;
        pr[2] = bb;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void solve_start_finish_kernel(SolveArgs<T> a, double tol2, double delta2,
                                                                 int maxit) {
    __shared__ double sh[4];
    const double *pr = part_rel(a.part);
    const double rz = sum_partials(pr, a.grid_vec, 3, sh);
    const double rr = sum_partials(pr + 1, a.grid_vec, 3, sh);
    const double bb = sum_partials(pr + 2, a.grid_vec, 3, sh);
    if (threadIdx.x == 0) {
        SolveScalars *S = a.sc;
        S->rz = rz;
        S->alpha = S->beta = 0.0;
        S->rr = rr;
        S->rr_max = rr;
        S->rr_true = bb;
        S->bb = bb;
        S->tol2 = tol2;
        S->delta2 = delta2;
        S->iter = 0;
        S->maxit = maxit;
        S->upd = 0;
        S->updates = 0;
        S->stalls = 0;
        S->broke = 0;
        S->done = (bb > 0.0 && rz > 0.0 && maxit > 0) ? 0 : 1;
    }
}

// q = L p; partial p.q per block
template <typename T, int G>
__global__ __launch_bounds__(256) void solve_spmv_kernel(SolveArgs<T> a, RowMap m) {
    __shared__ double sh[4];
    if (a.sc->done) return;  // uniform: written by an earlier kernel
    double acc = 0.0;
    T *__restrict__ q = a.q;
    const T *__restrict__ p = a.p;
    lap_apply_rows<T, G>(
        m, p,
        [&](int v, T qv) {
            q[v] = qv;
            acc += (double)p[v] * (double)qv;
        },
        blockIdx.x, gridDim.x);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part_pq(a.part)[blockIdx.x] = acc;
}

// alpha = z.r / p.q (one block); a breakdown (p.q not positive) ends the solve at the next update
template <typename T>
__global__ __launch_bounds__(256) void solve_alpha_kernel(SolveArgs<T> a) {
    __shared__ double sh[4];
    SolveScalars *S = a.sc;
    if (S->done) return;
    const double pq = sum_partials(part_pq(a.part), a.grid_spmv, 1, sh);
    if (threadIdx.x == 0) {
        if (pq > 0.0 && pq == pq) {
            S->alpha = S->rz / pq;
        } else {
            S->alpha = 0.0;
            S->broke = 1;
        }
    }
}

// xs += alpha p; rs -= alpha q; z = rs / diag; partials of z.r and r.r
template <typename T>
__global__ __launch_bounds__(256) void solve_update_kernel(SolveArgs<T> a) {
    __shared__ double sh[4];
    if (a.sc->done) return;
    const T al = (T)a.sc->alpha;
    double rz = 0.0, rr = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.xs[v] += al * a.p[v];
        const T rv = a.rs[v] - al * a.q[v];
        a.rs[v] = rv;
        const T zv = rv / jacobi_diag(a, v);
        a.z[v] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        double *pu = part_upd(a.part) + 2 * blockIdx.x;
        pu[0] = rz;
        pu[1] = rr;
    }
}

// one block: the iteration count, the reliable-update test, else beta
template <typename T>
__global__ __launch_bounds__(256) void solve_beta_kernel(SolveArgs<T> a) {
    __shared__ double sh[4];
    SolveScalars *S = a.sc;
    if (S->done) return;
    const double rzn = sum_partials(part_upd(a.part), a.grid_vec, 2, sh);
    const double rr = sum_partials(part_upd(a.part) + 1, a.grid_vec, 2, sh);
    if (threadIdx.x == 0) {
        S->iter += 1;
        S->rr = rr;
        const bool upd = S->broke || S->iter >= S->maxit || !(rr > S->tol2 * S->bb) || rr < S->delta2 * S->rr_max;
        if (rr > S->rr_max) S->rr_max = rr;
        S->upd = upd ? 1 : 0;
        if (!upd) {
            S->beta = S->rz != 0.0 ? rzn / S->rz : 0.0;
            S->rz = rzn;
        }
    }
}

// reliable update, part 1: x += xs, xs = 0
template <typename T>
__global__ __launch_bounds__(256) void solve_fold_kernel(SolveArgs<T> a) {
    if (!a.sc->upd) return;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.x[v] += (double)a.xs[v];
        a.xs[v] = (T)0;
    }
}

// reliable update, part 2: r = b - L x in FP64; rs = r; z = rs / diag; partials of z.r, r.r
template <typename T, int G>
__global__ __launch_bounds__(256) void solve_true_residual_kernel(SolveArgs<T> a, RowMap m) {
    __shared__ double sh[4];
    if (!a.sc->upd) return;
    const double inv_n = 1.0 / (double)a.n;
    double rz = 0.0, rt = 0.0;
    lap_apply_rows<double, G>(
        m, a.x,
        [&](int v, double lx) {
            const double rv = rhs_of(v, a.u, inv_n) - lx;
            const T rs = (T)rv;
            const T zv = rs / jacobi_diag(a, v);
            a.rs[v] = rs;
            a.z[v] = zv;
            rz += (double)rs * (double)zv;
            rt += rv * rv;
        },
        blockIdx.x, gridDim.x);
    rz = block_sum(rz, sh);
    rt = block_sum(rt, sh);
    if (threadIdx.x == 0) {
        double *pr = part_rel(a.part) + 2 * blockIdx.x;
        pr[0] = rz;
        pr[1] = rt;
    }
}

// reliable update, part 3 (one block): the true residual decides the end; else beta from the
// replaced residual.  Three updates in a row whose true residual fell by less than 2x
// (the rounding floor) also end the solve.
template <typename T>
__global__ __launch_bounds__(256) void solve_update_end_kernel(SolveArgs<T> a) {
    __shared__ double sh[4];
    SolveScalars *S = a.sc;
    if (!S->upd) return;
    const double rzn = sum_partials(part_rel(a.part), a.grid_spmv, 2, sh);
    const double rt = sum_partials(part_rel(a.part) + 1, a.grid_spmv, 2, sh);
    if (threadIdx.x == 0) {
        S->updates += 1;
        S->stalls = rt > 0.25 * S->rr_true ? S->stalls + 1 : 0;
        S->rr_true = rt;
        S->rr_max = rt;
        S->rr = rt;
        S->upd = 0;
        if (!(rt > S->tol2 * S->bb) || S->iter >= S->maxit || S->broke || S->stalls >= 3) {
            S->done = 1;
        } else {
            S->beta = S->rz != 0.0 ? rzn / S->rz : 0.0;
            S->rz = rzn;
        }
    }
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void solve_pdir_kernel(SolveArgs<T> a) {
    if (a.sc->done) return;
    const T be = (T)a.sc->beta;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x)
        a.p[v] = a.z[v] + be * a.p[v];
}

// ---------------------------------------------------------------------------------------
// the whole solve in one workgroup (small graphs, batch members): the same start, iteration,
// reliable updates and end rule, with no kernel boundary or host poll between iterations.
// Ends with the scalars the multi-kernel path leaves.
// ---------------------------------------------------------------------------------------
template <typename T, int G>
__device__ void solve_small_body(const SolveArgs<T> &a, const RowMap &m, double tol2, double delta2, int maxit,
                                 double *sh) {
    const int n = a.n, tid = threadIdx.x, u = a.u;
    const double inv_n = 1.0 / (double)n;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int v = tid; v < n; v += kSmallThreads) {
        const double b = rhs_of(v, u, inv_n);
        const T rv = (T)b;
        const T zv = rv / jacobi_diag(a, v);
        a.x[v] = 0.0;
        a.xs[v] = (T)0;
        a.rs[v] = rv;
        a.z[v] = zv;
        a.p[v] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
        bb += b * b;
    }
    rz = block_sum_t<double>(rz, sh);  // the barriers also publish p before the first product
    rr = block_sum_t<double>(rr, sh);
    bb = block_sum_t<double>(bb, sh);
    double rr_max = rr, rr_true = bb;
    int it = 0, updates = 0, stalls = 0;
    bool done = !(bb > 0.0 && rz > 0.0 && maxit > 0);
    while (!done) {
        double pq = 0.0;
        lap_apply_rows<T, G, kSmallThreads>(
            m, a.p,
            [&](int v, T qv) {
                a.q[v] = qv;
                pq += (double)a.p[v] * (double)qv;
            },
            0, 1);
        pq = block_sum_t<double>(pq, sh);
        const bool broke = !(pq > 0.0 && pq == pq);
        const T al = broke ? (T)0 : (T)(rz / pq);
        double rzn = 0.0, rrn = 0.0;
        for (int v = tid; v < n; v += kSmallThreads) {
            a.xs[v] += al * a.p[v];
            const T rv = a.rs[v] - al * a.q[v];
            a.rs[v] = rv;
            const T zv = rv / jacobi_diag(a, v);
            a.z[v] = zv;
            rzn += (double)rv * (double)zv;
            rrn += (double)rv * (double)rv;
        }
        rzn = block_sum_t<double>(rzn, sh);
        rrn = block_sum_t<double>(rrn, sh);
        ++it;
        const bool upd = broke || it >= maxit || !(rrn > tol2 * bb) || rrn < delta2 * rr_max;
        if (rrn > rr_max) rr_max = rrn;
        double beta;
        if (upd) {
            for (int v = tid; v < n; v += kSmallThreads) {
                a.x[v] += (double)a.xs[v];
                a.xs[v] = (T)0;
            }
            __syncthreads();  // x complete before the product gathers it
            double rz2 = 0.0, rt = 0.0;
            lap_apply_rows<double, G, kSmallThreads>(
                m, a.x,
                [&](int v, double lx) {
                    const double rv = rhs_of(v, u, inv_n) - lx;
                    const T rs = (T)rv;
                    const T zv = rs / jacobi_diag(a, v);
                    a.rs[v] = rs;
                    a.z[v] = zv;
                    rz2 += (double)rs * (double)zv;
                    rt += rv * rv;
                },
                0, 1);
            rz2 = block_sum_t<double>(rz2, sh);
            rt = block_sum_t<double>(rt, sh);
            ++updates;
            stalls = rt > 0.25 * rr_true ? stalls + 1 : 0;
            rr_true = rt;
            rr_max = rt;
            if (!(rt > tol2 * bb) || it >= maxit || broke || stalls >= 3) break;
            beta = rz != 0.0 ? rz2 / rz : 0.0;
            rz = rz2;
        } else {
            beta = rz != 0.0 ? rzn / rz : 0.0;
            rz = rzn;
        }
        const T be = (T)beta;
        for (int v = tid; v < n; v += kSmallThreads) a.p[v] = a.z[v] + be * a.p[v];
        __syncthreads();  // p complete before the next product gathers it
    }
    if (tid == 0) {
        SolveScalars *S = a.sc;
        S->rz = rz;
        S->rr = rr_true;
        S->rr_max = rr_max;
        S->rr_true = rr_true;
        S->bb = bb;
        S->tol2 = tol2;
        S->delta2 = delta2;
        S->iter = it;
        S->maxit = maxit;
        S->upd = 0;
        S->updates = updates;
        S->stalls = stalls;
        S->done = 1;
    }
}

template <typename T, int G>
__global__ __launch_bounds__(kSmallThreads) void solve_small_kernel(SolveArgs<T> a, RowMap m, double tol2,
                                                                    double delta2, int maxit) {
    __shared__ double sh[kSmallThreads / kWave];
    solve_small_body<T, G>(a, m, tol2, delta2, maxit, sh);
}

// independent solves side by side: workgroup i runs job i (one graph's pivot column)
template <typename T, int G>
__global__ __launch_bounds__(kSmallThreads) void solve_small_batch_kernel(const SolveJob<T> *__restrict__ jobs) {
    __shared__ double sh[kSmallThreads / kWave];
    const SolveJob<T> &j = jobs[blockIdx.x];
    solve_small_body<T, G>(j.a, j.m, j.tol2, j.delta2, j.maxit, sh);
}

// ---------------------------------------------------------------------------------------
// final residual and projection
// ---------------------------------------------------------------------------------------
// res = b - L x (nullable), per-block partials of [sum res, |res|^2, sum x]; reduce3_kernel
// sums them into out[0..3)
template <int G>
__global__ __launch_bounds__(256) void residual64_kernel(RowMap m, int u, const double *__restrict__ x,
                                                         double *__restrict__ res, double *__restrict__ part) {
    __shared__ double sh[4];
    const double inv_n = 1.0 / (double)m.n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    lap_apply_rows<double, G>(
        m, x,
        [&](int v, double lx) {
            const double rv = rhs_of(v, u, inv_n) - lx;
            if (res) res[v] = rv;
            s0 += rv;
            s1 += rv * rv;
            s2 += x[v];
        },
        blockIdx.x, gridDim.x);
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3] = s0;
        part[blockIdx.x * 3 + 1] = s1;
        part[blockIdx.x * 3 + 2] = s2;
    }
}

__global__ __launch_bounds__(256) void reduce3_kernel(const double *__restrict__ part, int nparts,
                                                      double *__restrict__ out) {
    __shared__ double sh[4];
    const double a0 = sum_partials(part, nparts, 3, sh);
    const double a1 = sum_partials(part + 1, nparts, 3, sh);
    const double a2 = sum_partials(part + 2, nparts, 3, sh);
    if (threadIdx.x == 0) {
        out[0] = a0;
        out[1] = a1;
        out[2] = a2;
    }
}

// x -= mean_src[0] / n (mean-zero projection)
__global__ __launch_bounds__(256) void project_kernel(int n, double *__restrict__ x,
                                                     const double *__restrict__ mean_src) {
    const double mean = mean_src[0] / (double)n;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) x[v] -= mean;
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
int solve_grid(const RowMap &m, int G) {
    const long long tiles = ((long long)m.n + (256 / G) - 1) / (256 / G);
    return (int)std::min<long long>(std::max<long long>(tiles, 1), kMaxSolveGrid);
}
int vec_grid(int n) { return std::max(1, std::min((n + 255) / 256, kMaxSolveGrid)); }

template <typename T>
hipError_t launch_solve_start(const SolveArgs<T> &a, double tol2, double delta2, int maxit, hipStream_t st) {
    solve_start_kernel<T><<<a.grid_vec, 256, 0, st>>>(a);
    solve_start_finish_kernel<T><<<1, 256, 0, st>>>(a, tol2, delta2, maxit);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_solve_iteration(const SolveArgs<T> &a, const RowMap &m, int G, hipStream_t st) {
    USTD_DISPATCH_G(G, (solve_spmv_kernel<T, GG><<<a.grid_spmv, 256, 0, st>>>(a, m)));
    solve_alpha_kernel<T><<<1, 256, 0, st>>>(a);
    solve_update_kernel<T><<<a.grid_vec, 256, 0, st>>>(a);
    solve_beta_kernel<T><<<1, 256, 0, st>>>(a);
    solve_fold_kernel<T><<<a.grid_vec, 256, 0, st>>>(a);
    USTD_DISPATCH_G(G, (solve_true_residual_kernel<T, GG><<<a.grid_spmv, 256, 0, st>>>(a, m)));
    solve_update_end_kernel<T><<<1, 256, 0, st>>>(a);
    solve_pdir_kernel<T><<<a.grid_vec, 256, 0, st>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_solve_small(const SolveArgs<T> &a, const RowMap &m, int G, double tol2, double delta2, int maxit,
                              hipStream_t st) {
    USTD_DISPATCH_G(G, (solve_small_kernel<T, GG><<<1, kSmallThreads, 0, st>>>(a, m, tol2, delta2, maxit)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_solve_small_batch(const SolveJob<T> *jobs, int count, int G, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    USTD_DISPATCH_G(G, (solve_small_batch_kernel<T, GG><<<count, kSmallThreads, 0, st>>>(jobs)));
    return hipGetLastError();
}

#define USTD_SOLVE_INSTANTIATE(T)                                                                              \
    template hipError_t launch_solve_start<T>(const SolveArgs<T> &, double, double, int, hipStream_t);         \
    template hipError_t launch_solve_iteration<T>(const SolveArgs<T> &, const RowMap &, int, hipStream_t);     \
    template hipError_t launch_solve_small<T>(const SolveArgs<T> &, const RowMap &, int, double, double, int,  \
                                              hipStream_t);                                                    \
    template hipError_t launch_solve_small_batch<T>(const SolveJob<T> *, int, int, hipStream_t);
USTD_SOLVE_INSTANTIATE(double)
USTD_SOLVE_INSTANTIATE(float)
#undef USTD_SOLVE_INSTANTIATE

hipError_t launch_residual64(const RowMap &m, int G, int u, const double *x, double *res, double *part, double *out,
                             hipStream_t st) {
    const int grid = solve_grid(m, G);
    USTD_DISPATCH_G(G, residual64_kernel<GG><<<grid, 256, 0, st>>>(m, u, x, res, part));
    reduce3_kernel<<<1, 256, 0, st>>>(part, grid, out);
    return hipGetLastError();
}

hipError_t launch_project(int n, double *x, const double *mean_src, int grid, hipStream_t st) {
    project_kernel<<<grid, 256, 0, st>>>(n, x, mean_src);
    return hipGetLastError();
}

}  // namespace ustd
