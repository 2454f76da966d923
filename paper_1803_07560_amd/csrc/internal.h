// Internal interface between the host runtime (runtime.cpp) and the per-shape
// kernel translation units (shape_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfi {

// Lattice shapes with compiled kernels, as (nx, nt) = (space sites, time slices).
#define BFI_SHAPES(X)                                                                   \
    X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(4, 2) X(5, 3) X(8, 2)     \
    X(10, 2) X(16, 4)

// kFP64: plain weights exp(-S); kFP32Shifted: FP32 action and exp with a
// per-thread shift; kFP64Shifted: FP64 action and exp with a per-thread shift.
enum Precision : int { kFP64 = 0, kFP32Shifted = 1, kFP64Shifted = 2 };

// Coefficients of the residual rewritten as
//   R = v_next + v (k_diag + c_adv (v_right - v_left)) - c_visc (v_right + v_left)
// with c_adv = g tau / (2a), c_visc = nu tau / a^2, k_diag = 2 c_visc - 1;
// S = inv_2Dtau * sum R^2 + half_m2 * sum u^2.
struct ActionCoef {
    double k_diag, c_adv, c_visc, inv_2Dtau, half_m2;
};

// Everything one evaluation (a plan, or one served request) shares, resident in
// device memory: the subvolumes' point maps, Philox ids and first sample
// indices, the action coefficients and the seed.
struct EvalParams {
    const double *base64, *scale64;  // nsub x d: point map in FP64
    const float *base32, *scale32;   // nsub x d: point map in FP32
    const uint64_t *ids;             // nsub heap ids (Philox counter words 2-3)
    const uint64_t *offsets;         // nsub first sample index
    ActionCoef coef;
    uint32_t seed_lo, seed_hi;
};

// One unit of device work: `count` consecutive samples of subvolume `sub` of
// `params`, starting `start` samples after the subvolume's own offset; the
// item's partial record goes to `rec` (4 + 3 nx doubles).  Every item of one
// launch shares the lattice shape, the precision and the observable.
struct WorkItem {
    const EvalParams *params;
    double *rec;
    uint64_t start;
    uint32_t sub;
    uint32_t count;
};

struct McArgs {
    const WorkItem *items;   // nitems
    double *item_split;      // nitems x 2d (split statistics), or null
    uint32_t *queue_head;    // persistent kernels: next item to take
    uint32_t nitems;
    uint32_t samples_per_thread;
};

// Block sizes the Monte Carlo kernels are compiled for (split statistics:
// 256 only).
inline bool mc_block_ok(int block)
{
    return block == 64 || block == 128 || block == 256 || block == 512 || block == 1024;
}

struct LaunchSpec {
    int prec;        // Precision
    int block;       // 64, 128, 256, 512, 1024
    int split;       // 0/1
    int persistent;  // 0/1
    uint32_t grid;   // blocks
    int obs = 0;     // bfi_observable: 0 anchored product, 1 averaged over anchors
    int pair = 0;    // 1: antithetic pairs (d <= kMaxPairD, no split statistics)
};

// Largest lattice the antithetic-pair kernels are compiled for.
constexpr int kMaxPairD = 32;

struct MergeArgs {
    const double *item_rec;     // nitems x rec_len
    const double *item_split;   // nitems x 2d or null
    const uint32_t *sub_first;  // nsub + 1 prefix of item indices
    double *sub_rec;            // nsub x rec_len
    double *sub_split;          // nsub x (1 + 2d) or null
    uint32_t nsub;
    int32_t nx, d;
};

struct DebugPointArgs {
    const double *base64, *scale64;  // d each
    const float *base32, *scale32;   // d each
    const uint64_t *index;           // n sample indices
    double *out;                     // n x d
    uint64_t id;
    uint64_t n;
    uint32_t seed_lo, seed_hi;
    int32_t d;
    int32_t prec;
};

struct DebugActionArgs {
    const double *points;  // n x d
    double *out;           // n
    uint64_t n;
    ActionCoef coef;
    int32_t prec;
};

struct KernelInfo {
    int vgprs, sgprs, blocks_per_cu;
};

template <int NX, int NT>
hipError_t launch_mc_shape(const LaunchSpec &spec, const McArgs &args, hipStream_t stream);
template <int NX, int NT>
hipError_t kernel_info_shape(const LaunchSpec &spec, KernelInfo *info);
template <int NX, int NT>
hipError_t launch_debug_action_shape(const DebugActionArgs &args, hipStream_t stream);

#define BFI_DECLARE_SHAPE(NX, NT)                                                        \
    extern template hipError_t launch_mc_shape<NX, NT>(const LaunchSpec &, const McArgs &, \
                                                       hipStream_t);                     \
    extern template hipError_t kernel_info_shape<NX, NT>(const LaunchSpec &, KernelInfo *); \
    extern template hipError_t launch_debug_action_shape<NX, NT>(const DebugActionArgs &,  \
                                                                 hipStream_t);
BFI_SHAPES(BFI_DECLARE_SHAPE)
#undef BFI_DECLARE_SHAPE

// N-sphere test integrand f(x) = sqrt(1 - |x|^2) (0 outside the unit ball) over
// boxes of `dim` <= kMaxNsphereDim dimensions, FP64.  Records follow the Burgers
// layout with nx = 0: [n, 0, sum f, sum f^2]; split statistics [sum_U f (dim),
// sum_U f^2 (dim)] per item.  Blocks of 256 threads.
constexpr int kMaxNsphereDim = 16;
struct NsphereArgs {
    McArgs mc;
    int32_t dim;
};

// Work items and point maps built on the device from a copied subvolume list
// (n, lo, hi): sub_first[s] = first item of subvolume s (nsub + 1 entries, a
// prefix sum of ceil(n_s / chunk)), then per subvolume the FP64 and FP32 maps
// (scale = (hi - lo) 2^-32, base = lo + scale/2, as the host computes them) and
// items of `chunk` consecutive samples whose records go to item_rec.
struct BuildArgs {
    const double *lo, *hi;
    const uint64_t *n;
    uint32_t *sub_first;
    double *base64, *scale64;
    float *base32, *scale32;
    WorkItem *items;
    const EvalParams *params;
    double *item_rec;
    uint64_t chunk;
    uint32_t nsub;
    int32_t d, rec_len;
};

// Leaf records of an adaptive run kept in device memory (leaf_kernels.hip).
// Record layouts are those of bfi_eval: per leaf a partial record of the
// Burgers layout (4 + 3 nx doubles: count, shift, sums), split statistics
// (1 + 2d: shift, upper-half sums) and the record of the samples the split
// statistics cover, plus the leaf's volume.
//
// Fold: a round's entries into the leaves.  Entry e's records are the rows
// wpos (split-statistics pass: record and split statistics) and opos (plain
// pass), -1 where it has no samples there; kind 0 merges them into leaf dst
// (a doubled leaf continuing its stream), kinds 1 and 2 write leaf dst (the
// children of a split leaf; vol is the child's volume).
struct FoldEntry {
    uint32_t dst;
    int32_t kind;
    int32_t wpos, opos;
    double vol;
};
struct FoldArgs {
    const FoldEntry *entries;
    uint32_t count;
    const double *with_rec, *with_split, *plain_rec;
    double *leaf_rec, *leaf_split, *leaf_base, *leaf_vol;
    int32_t nx, d;
};
hipError_t launch_fold(const FoldArgs &args, hipStream_t stream);

// Analysis of every leaf for the adaptive driver, as bfi_finalize's two passes
// over the records and the driver's split choice: the common shift (smallest
// sigma), the totals of the first pass (Z, Var Z, sum of squared weights,
// samples, N(r)), then per leaf its contribution e to the variance of C
// (clamped at 0, NaN as 0), the dimension j* minimising sigma_lower +
// sigma_upper of its split statistics and the gain (sigma_L + sigma_U)(j*) /
// (2 sigma), and the totals of the second pass (the variance of C(r) before
// the division by Z^2).  Per-block sums in a fixed tree order, the blocks'
// sums in block order with Neumaier compensation: the result does not depend
// on timing.  out_totals (host-visible) gets [sigma, 4 + nx first-pass totals,
// nx second-pass totals]; e, best and gain one value per leaf.
constexpr int kAnalysisBlock = 1024;
constexpr int kMaxAnalysisNx = 32;
struct LeafAnalysisArgs {
    const double *rec, *split, *base, *vol;
    uint32_t count;
    int32_t nx, d;
    double *scratch;     // analysis_scratch_doubles(count, nx) doubles
    double *out_totals;  // 1 + 4 + 2 nx doubles
    double *e, *gain;    // count each
    int32_t *best;       // count
};
size_t analysis_scratch_doubles(uint32_t count, int nx);
hipError_t launch_leaf_analysis(const LeafAnalysisArgs &args, hipStream_t stream);

// Shape-independent kernels (common_kernels.hip).
hipError_t launch_build_items(const BuildArgs &args, hipStream_t stream);
hipError_t launch_reset_head(uint32_t *head, hipStream_t stream);
hipError_t launch_nsphere(const NsphereArgs &args, uint32_t grid, hipStream_t stream);
hipError_t launch_merge(const MergeArgs &args, hipStream_t stream);
hipError_t launch_debug_points(const DebugPointArgs &args, hipStream_t stream);

}  // namespace bfi
