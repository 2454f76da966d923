// Leaf records of an adaptive run in device memory: the fold of a round's
// records into the leaves and the analysis of every leaf (the finalize's two
// passes over the records, paper section 2's estimators of Z and C(r) with
// their delta-method errors, and the refinement's split choice, section 3).
// The arithmetic is the host's (finalize_records, merge_shifted, split_choice)
// operation for operation, without contraction into fused multiply-adds; only
// the order of the sums over leaves differs (tree sums per block, blocks in
// order with Neumaier compensation).
#include "device.hpp"

#pragma clang fp contract(off)

namespace bfi {
namespace {

// Field classes of a record: 0 the count, 1 the shift, 2 first-order sums
// (scaled by the shift factor), 3 second-order sums (by its square).
__device__ __forceinline__ int rec_class(int f, int nx)
{
    return f == 0 ? 0 : f == 1 ? 1 : f == 2 ? 2 : f == 3 ? 3 : f < 4 + nx ? 2 : 3;
}
// Split statistics: the shift, then d first-order and d second-order sums.
__device__ __forceinline__ int split_class(int f, int d)
{
    return f == 0 ? 1 : f <= d ? 2 : 3;
}

// a <- a merged with b (disjoint samples of one leaf), both moved to the
// smaller shift; counts add where there is a count.
__device__ void merge_into(double *a, const double *b, int len, bool is_split, int nx, int d)
{
    const int sa = is_split ? 0 : 1;
    const double sig = b[sa] < a[sa] ? b[sa] : a[sa];
    const double fa = exp(sig - a[sa]), fb = exp(sig - b[sa]);
    for (int f = 0; f < len; ++f) {
        const int c = is_split ? split_class(f, d) : rec_class(f, nx);
        if (c == 2)
            a[f] = fa * a[f] + fb * b[f];
        else if (c == 3)
            a[f] = fa * fa * a[f] + fb * fb * b[f];
        else if (c == 0)
            a[f] += b[f];
    }
    a[sa] = sig;
}

// The record of an entry's samples from its two parts (either may be absent),
// written to out: the first part, then the second merged in (a part with no
// samples adds nothing).
__device__ void combine_parts(double *out, const double *w, const double *p, int rec_len, int nx,
                              int d)
{
    if (w)
        for (int f = 0; f < rec_len; ++f)
            out[f] = w[f];
    else
        for (int f = 0; f < rec_len; ++f)
            out[f] = 0.0;
    if (!p || p[0] == 0)
        return;
    if (out[0] == 0) {
        for (int f = 0; f < rec_len; ++f)
            out[f] = p[f];
        return;
    }
    merge_into(out, p, rec_len, false, nx, d);
}

constexpr int kFoldBlock = 128;
constexpr int kMaxRecLen = 4 + 3 * kMaxAnalysisNx;

// One thread per entry; every entry has a leaf of its own.
__global__ void __launch_bounds__(kFoldBlock) fold_kernel(FoldArgs a)
{
    const uint32_t i = blockIdx.x * kFoldBlock + threadIdx.x;
    if (i >= a.count)
        return;
    const FoldEntry en = a.entries[i];
    const int nx = a.nx, d = a.d, rec_len = 4 + 3 * nx, split_len = 1 + 2 * d;
    const double *w = en.wpos >= 0 ? a.with_rec + static_cast<size_t>(en.wpos) * rec_len : nullptr;
    const double *sp =
        en.wpos >= 0 ? a.with_split + static_cast<size_t>(en.wpos) * split_len : nullptr;
    const double *p = en.opos >= 0 ? a.plain_rec + static_cast<size_t>(en.opos) * rec_len : nullptr;
    double *lrec = a.leaf_rec + static_cast<size_t>(en.dst) * rec_len;
    double *lsplit = a.leaf_split + static_cast<size_t>(en.dst) * split_len;
    double *lbase = a.leaf_base + static_cast<size_t>(en.dst) * rec_len;
    if (en.kind == 0) {
        double R[kMaxRecLen];
        combine_parts(R, w, p, rec_len, nx, d);
        merge_into(lrec, R, rec_len, false, nx, d);
        if (w && w[0] > 0) {
            // the continuation still lies below the split statistics' cut
            merge_into(lsplit, sp, split_len, true, nx, d);
            merge_into(lbase, w, rec_len, false, nx, d);
        }
        return;
    }
    combine_parts(lrec, w, p, rec_len, nx, d);
    for (int f = 0; f < split_len; ++f)
        lsplit[f] = sp ? sp[f] : 0.0;
    for (int f = 0; f < rec_len; ++f)
        lbase[f] = w ? w[f] : 0.0;
    a.leaf_vol[en.dst] = en.vol;
}

// ---- analysis ----------------------------------------------------------------

// scratch layout (doubles): per block the smallest shift, the first pass's
// 4 + nx sums and the second pass's nx sums; then [sigma, z, 1/z^2, C(r)]
__device__ __forceinline__ size_t nblocks_of(uint32_t count)
{
    return (static_cast<size_t>(count) + kAnalysisBlock - 1) / kAnalysisBlock;
}

// A block's sums of several terms in a fixed order: each term's wavefront
// butterflies (wave_part), then, after one barrier, thread j adds term j's
// wave sums in wave order (block_parts_out).
constexpr int kAnalysisWaves = kAnalysisBlock / 64;
__device__ __forceinline__ void wave_part(double v, double (*lds)[kAnalysisWaves], int j)
{
    const double s = dev::wave_sum(v);
    if ((threadIdx.x & 63) == 0)
        lds[j][threadIdx.x >> 6] = s;
}
__device__ __forceinline__ void block_parts_out(const double (*lds)[kAnalysisWaves], int count,
                                                double *part)
{
    if (static_cast<int>(threadIdx.x) < count) {
        double t = 0.0;
        for (int k = 0; k < kAnalysisWaves; ++k)
            t += lds[threadIdx.x][k];
        part[threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kAnalysisBlock) shift_kernel(LeafAnalysisArgs a)
{
    __shared__ double m[kAnalysisBlock];
    const uint32_t s = blockIdx.x * kAnalysisBlock + threadIdx.x;
    const int rec_len = 4 + 3 * a.nx;
    m[threadIdx.x] = s < a.count ? a.rec[static_cast<size_t>(s) * rec_len + 1] : __builtin_inf();
    __syncthreads();
    for (int k = kAnalysisBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            const double x = m[threadIdx.x + k];
            // the smaller of the two, a NaN never taken (the host's std::min)
            if (x < m[threadIdx.x])
                m[threadIdx.x] = x;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        a.scratch[blockIdx.x] = m[0];
}

__global__ void __launch_bounds__(kAnalysisBlock) shift_reduce_kernel(LeafAnalysisArgs a)
{
    __shared__ double m[kAnalysisBlock];
    const size_t nb = nblocks_of(a.count);
    const int nx = a.nx;
    double *scal = a.scratch + nb * (1 + 4 + 2 * nx);
    double sig = __builtin_inf();
    for (size_t b = threadIdx.x; b < nb; b += kAnalysisBlock)
        if (a.scratch[b] < sig)
            sig = a.scratch[b];
    m[threadIdx.x] = sig;
    __syncthreads();
    for (int k = kAnalysisBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k && m[threadIdx.x + k] < m[threadIdx.x])
            m[threadIdx.x] = m[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[0] = m[0];
        a.out_totals[0] = m[0];
    }
}

__global__ void __launch_bounds__(kAnalysisBlock) first_pass_kernel(LeafAnalysisArgs a)
{
    __shared__ double lds[4 + kMaxAnalysisNx][kAnalysisWaves];
    const size_t nb = nblocks_of(a.count);
    const int nx = a.nx, rec_len = 4 + 3 * nx, nt = 4 + nx;
    const double sig = a.scratch[nb * (1 + 4 + 2 * nx)];
    const uint32_t s = blockIdx.x * kAnalysisBlock + threadIdx.x;
    const bool on = s < a.count;
    const double *rec = a.rec + static_cast<size_t>(on ? s : 0) * rec_len;
    double n = 1.0, vol = 0.0, aa = 0.0, sw = 0.0, sw2 = 0.0;
    if (on) {
        n = rec[0];
        vol = a.vol[s];
        aa = exp(sig - rec[1]);
        sw = aa * rec[2];
        sw2 = aa * aa * rec[3];
    }
    double *part = a.scratch + nb + static_cast<size_t>(blockIdx.x) * nt;
    // the finalize's sums: Z, Var Z, squared weights, samples, N(r)
    for (int j = 0; j < nt; ++j) {
        double t = 0.0;
        if (on) {
            if (j == 0)
                t = vol * sw / n;
            else if (j == 1)
                t = vol * vol * (sw2 - sw * sw / n) / (n * (n - 1.0));
            else if (j == 2)
                t = (vol / n) * (vol / n) * sw2;
            else if (j == 3)
                t = n;
            else
                t = vol * aa * rec[j] / n;
        }
        wave_part(t, lds, j);
    }
    __syncthreads();
    block_parts_out(lds, nt, part);
}

// Neumaier sum of the blocks' partial sums in block order; thread j takes sum
// j.  Loads go eight at a time ahead of their additions.
__device__ double ordered_total(const double *part, size_t nb, int stride, int j)
{
    constexpr size_t kBatch = 8;
    double sum = 0.0, comp = 0.0;
    for (size_t b0 = 0; b0 < nb; b0 += kBatch) {
        double xb[kBatch];
#pragma unroll
        for (size_t k = 0; k < kBatch; ++k)
            xb[k] = b0 + k < nb ? part[(b0 + k) * stride + j] : 0.0;
#pragma unroll
        for (size_t k = 0; k < kBatch; ++k) {
            if (b0 + k < nb) {
                const double x = xb[k];
                const double t = sum + x;
                comp += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
                sum = t;
            }
        }
    }
    return sum + comp;
}

__global__ void __launch_bounds__(64) first_reduce_kernel(LeafAnalysisArgs a)
{
    __shared__ double tot[4 + kMaxAnalysisNx];
    const size_t nb = nblocks_of(a.count);
    const int nx = a.nx, nt = 4 + nx;
    double *scal = a.scratch + nb * (1 + 4 + 2 * nx);
    for (int j = threadIdx.x; j < nt; j += 64) {
        tot[j] = ordered_total(a.scratch + nb, nb, nt, j);
        a.out_totals[1 + j] = tot[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double z = tot[0];
        scal[1] = z;
        scal[2] = z > 0 ? 1.0 / (z * z) : 0.0;
        for (int r = 0; r < nx; ++r)
            scal[3 + r] = tot[4 + r] / z;
    }
}

// The leaf's split choice from its split statistics and the record of the
// samples they cover (the host's split_choice).
__device__ void split_choice(const double *sp, const double *base, int d, int32_t *best_out,
                             double *gain_out)
{
    const double S = base[2], Q = base[3], m = base[0], half = 0.5 * m;
    const double v = Q / m - (S / m) * (S / m);
    const double sigma = sqrt(v < 0.0 ? 0.0 : v);
    double best = __builtin_inf();
    int best_j = 0;
    for (int j = 0; j < d; ++j) {
        const double su = sp[1 + j], qu = sp[1 + d + j];
        const double sl = S - su, ql = Q - qu;
        const double vu0 = qu / half - (su / half) * (su / half);
        const double vl0 = ql / half - (sl / half) * (sl / half);
        const double vu = vu0 < 0.0 ? 0.0 : vu0, vl = vl0 < 0.0 ? 0.0 : vl0;
        const double sj = sqrt(vu) + sqrt(vl);
        if (sj < best) {
            best = sj;
            best_j = j;
        }
    }
    *best_out = best_j;
    *gain_out = sigma > 0 ? best / (2.0 * sigma) : 1.0;
}

__global__ void __launch_bounds__(kAnalysisBlock) second_pass_kernel(LeafAnalysisArgs a)
{
    __shared__ double lds[kMaxAnalysisNx][kAnalysisWaves];
    const size_t nb = nblocks_of(a.count);
    const int nx = a.nx, d = a.d, rec_len = 4 + 3 * nx, split_len = 1 + 2 * d;
    const double *scal = a.scratch + nb * (1 + 4 + 2 * nx);
    const double sig = scal[0], inv_z2 = scal[2];
    const uint32_t s = blockIdx.x * kAnalysisBlock + threadIdx.x;
    const bool on = s < a.count;
    const double *rec = a.rec + static_cast<size_t>(on ? s : 0) * rec_len;
    double *part = a.scratch + nb * (1 + 4 + nx) + static_cast<size_t>(blockIdx.x) * nx;
    double n = 1.0, v2 = 0.0, nn = 1.0, aa = 0.0, a2 = 0.0, sw = 0.0, var_z = 0.0;
    if (on) {
        n = rec[0];
        const double vol = a.vol[s];
        v2 = vol * vol;
        nn = n * (n - 1.0);
        aa = exp(sig - rec[1]);
        a2 = aa * aa;
        sw = aa * rec[2];
        const double sw2 = a2 * rec[3];
        var_z = v2 * (sw2 - sw * sw / n) / nn;
    }
    double e = 0.0;
    for (int r = 0; r < nx; ++r) {
        double t = 0.0;
        if (on) {
            const double C = scal[3 + r];
            const double spw = aa * rec[4 + r], spw2 = a2 * rec[4 + nx + r],
                         spww = a2 * rec[4 + 2 * nx + r];
            const double var_n = v2 * (spw2 - spw * spw / n) / nn;
            const double cov = v2 * (spww - spw * sw / n) / nn;
            t = var_n - 2.0 * C * cov + C * C * var_z;
            e += t;
        }
        wave_part(t, lds, r);
    }
    __syncthreads();
    block_parts_out(lds, nx, part);
    if (!on)
        return;
    // the host's max(e, 0) / Z^2, read back as a contribution (NaN counts 0)
    const double c = (e < 0.0 ? 0.0 : e) * inv_z2;
    a.e[s] = c >= 0.0 ? c : 0.0;
    split_choice(a.split + static_cast<size_t>(s) * split_len,
                 a.base + static_cast<size_t>(s) * rec_len, d, &a.best[s], &a.gain[s]);
}

__global__ void __launch_bounds__(64) second_reduce_kernel(LeafAnalysisArgs a)
{
    const size_t nb = nblocks_of(a.count);
    const int nx = a.nx;
    for (int r = threadIdx.x; r < nx; r += 64)
        a.out_totals[1 + 4 + nx + r] = ordered_total(a.scratch + nb * (1 + 4 + nx), nb, nx, r);
}

}  // namespace

hipError_t launch_fold(const FoldArgs &args, hipStream_t stream)
{
    if (args.count == 0)
        return hipSuccess;
    if (args.nx < 1 || args.nx > kMaxAnalysisNx || args.d < 1 || args.d > 32)
        return hipErrorInvalidValue;
    const uint32_t grid = (args.count + kFoldBlock - 1) / kFoldBlock;
    hipLaunchKernelGGL(fold_kernel, dim3(grid), dim3(kFoldBlock), 0, stream, args);
    return hipGetLastError();
}

size_t analysis_scratch_doubles(uint32_t count, int nx)
{
    const size_t nb = (static_cast<size_t>(count) + kAnalysisBlock - 1) / kAnalysisBlock;
    return nb * (1 + 4 + 2 * static_cast<size_t>(nx)) + 3 + static_cast<size_t>(nx);
}

hipError_t launch_leaf_analysis(const LeafAnalysisArgs &args, hipStream_t stream)
{
    if (args.count == 0 || args.nx < 1 || args.nx > kMaxAnalysisNx || args.d < 1 || args.d > 32)
        return hipErrorInvalidValue;
    const uint32_t grid = static_cast<uint32_t>(
        (static_cast<size_t>(args.count) + kAnalysisBlock - 1) / kAnalysisBlock);
    hipLaunchKernelGGL(shift_kernel, dim3(grid), dim3(kAnalysisBlock), 0, stream, args);
    hipLaunchKernelGGL(shift_reduce_kernel, dim3(1), dim3(kAnalysisBlock), 0, stream, args);
    hipLaunchKernelGGL(first_pass_kernel, dim3(grid), dim3(kAnalysisBlock), 0, stream, args);
    hipLaunchKernelGGL(first_reduce_kernel, dim3(1), dim3(64), 0, stream, args);
    hipLaunchKernelGGL(second_pass_kernel, dim3(grid), dim3(kAnalysisBlock), 0, stream, args);
    hipLaunchKernelGGL(second_reduce_kernel, dim3(1), dim3(64), 0, stream, args);
    return hipGetLastError();
}

}  // namespace bfi
