// Internal declarations shared by the host plan code (plan.cpp) and the
// device kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fastsum {

constexpr int kBlock = 256;        // threads per workgroup for every kernel
constexpr int kMaxPairs = 4;       // W/2 for W <= 8
constexpr int kMaxHalfCoef = 4;    // coefficients per even/odd half-polynomial

// Window weights of one point as polynomials of sp = frac(u) - 1/2, where u
// is the point's position in grid cells.  Tap t (t < W/2) and its mirror tap
// W-1-t share an even part E_t(sp^2) and an odd part sp*O_t(sp^2):
//   weight_t = E_t + sp O_t,   weight_{W-1-t} = E_t - sp O_t.
struct WindowArgs {
    float even[kMaxPairs][kMaxHalfCoef];
    float odd[kMaxPairs][kMaxHalfCoef];
};

// Grid geometry: n cells, position u = x~ * n + n/2 for x~ in [-1/2, 1/2).
// Only cells [lo, lo + nr) can receive or serve weight for points inside the
// plan's bound; the kernels clamp every point's taps into that range.
struct GridGeom {
    int n;
    int lo;
    int nr;
};

// Bound of App. J, eq. radius_xy: every pair difference stays inside the
// period of the rescaled kernel only if max ||x|| + max ||y|| <= R.  The
// kernels that read the points (operand-tile writers, projection GEMMs)
// record the largest |z / R|^2 of their rows as float bits (non-finite rows
// record +inf) into the norm slots of a role (0 sources, 1 targets); the
// last kernel of an exec compares sqrt(max role 0) + sqrt(max role 1) (role
// 0 twice when the targets are the sources) with lim, sets *flag when the
// sum is larger (or not finite) and clears every slot.  A role has
// kNormSlots slots on separate 64-byte lines, picked by workgroup, so the
// atomics of thousands of waves do not queue on one address.
constexpr int kNormSlots = 64;
constexpr int kNormStride = 16;                              // unsigned ints
constexpr int kNormRoleUints = kNormSlots * kNormStride;
constexpr int kNormUints = 2 * kNormRoleUints;               // both roles

struct BoundCheck {
    unsigned* norms;   // kNormUints slots; nullptr: no check in this launch
    int* flag;
    float lim;         // (1 + 1e-5) / max_p |xi_p|
    int same;          // targets are the sources: role 0 holds both
};

// Running max of squared row norms of a wave (every lane active) into the
// role's slot of this workgroup (role = norms of one role).
__device__ inline void record_norm2(unsigned* role, float n2) {
    unsigned u = (n2 <= 3.4e38f) ? __float_as_uint(n2) : 0x7f800000u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) u = max(u, (unsigned)__shfl_xor((int)u, o));
    if ((threadIdx.x & 63) == 0) atomicMax(role + (blockIdx.x % kNormSlots) * kNormStride, u);
}

__device__ inline unsigned wave_max_u32(unsigned u) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) u = max(u, (unsigned)__shfl_xor((int)u, o));
    return u;
}

// One full wave (64 lanes, kNormSlots == 64): the comparison and the reset
// described at BoundCheck.
__device__ inline void finish_bound_check(const BoundCheck& bc) {
    if (bc.norms == nullptr) return;
    const int lane = threadIdx.x & 63;
    unsigned* s0 = bc.norms + lane * kNormStride;
    unsigned* s1 = s0 + kNormRoleUints;
    const unsigned ua = wave_max_u32(*s0), ub = wave_max_u32(*s1);
    const float a = sqrtf(__uint_as_float(ua));
    const float b = bc.same ? a : sqrtf(__uint_as_float(ub));
    if (lane == 0 && !(a + b <= bc.lim)) atomicOr(bc.flag, 1);
    *s0 = 0u;
    *s1 = 0u;
}

// ---- launchers (kernels.hip); all asynchronous on `stream` ----

// clears the kNormUints norm slots (a fill kernel, so a graph capture
// records no memset)
hipError_t launch_clear_norms(unsigned* norms, hipStream_t stream);
// largest |x_n * scale|^2 over the rows of X (N x d) into the slots of
// `role`, one wave per row
hipError_t launch_point_norms(const float* X, int64_t N, int d, float scale, unsigned* role,
                              hipStream_t stream);

// out[p*ld + j] = sum_i A[p*dpad + i] * X[j*d + i] for p < P, j < N, with
// A = tau * Xi^T.  Sets *flag if |out| > bound.  norm_slot (nullable):
// largest |x_n * inv_r|^2, see BoundCheck.
// FP32 MFMA, d <= 64: A64 is A zero-padded to round_up(P, 64) x 64.
constexpr int kA64Cols = 64;
hipError_t launch_project_f32(const float* X, int64_t N, int d, const float* A64, int P,
                              float* out, int64_t ld, float bound, int* flag,
                              unsigned* norm_slot, float inv_r, hipStream_t stream);
// Tile GEMM, any d: X is first written as operand tiles into xtiles (the
// tile layout of the fused path below; bf16: one BF16 part per k-block,
// else f16 hi + lo of x * inv_r), then multiplied with the direction tiles
// At (bf16: BF16 tau xi; else f16 hi + lo of xi); out = pscale * product.
// The split form has FP32-level accuracy.
size_t project_tiles_bytes(int64_t rows, int d, bool bf16);
// Back-projection on the tile GEMM (d above the fused range):
// grad[m * d + i] = coef v[m] sum_p T[p * ld + m] tau xi_p[i], T: P x M.
// xit: split tiles of xi^T (rows i, columns p; xi_transpose_tiles_host);
// ttiles: backproject_tiles_bytes(M, P) bytes of scratch; scratch:
// backproject_scratch_bytes() bytes.
size_t backproject_tiles_bytes(int64_t rows, int P);
size_t backproject_scratch_bytes();
hipError_t launch_backproject_tiles(const float* T, int64_t ld, int64_t M, int P, int d,
                                    const uint16_t* xit, float tau, float coef, const float* v,
                                    float* grad, uint16_t* ttiles, void* scratch,
                                    hipStream_t stream);
hipError_t launch_project_tiles(const float* X, int64_t N, int d, bool bf16, const uint16_t* At,
                                int P, float inv_r, float pscale, uint16_t* xtiles, float* out,
                                int64_t ld, float bound, int* flag, unsigned* norm_slot,
                                hipStream_t stream);

// partial[(c*P + p)*nr + j - lo] = sum over sources i of chunk c of
//   w[i] * window(cell j - u(proj[p*ld + i]))
// chunk_len must be a multiple of kSliceLen; slice_max is scratch for
// ceil(N / kSliceLen) floats.
constexpr int kSliceLen = 4096;
hipError_t launch_spread(int W, const float* proj, int64_t ld, const float* w,
                         int64_t N, int P, GridGeom g, int nchunk,
                         int64_t chunk_len, float* slice_max, const WindowArgs& win,
                         float* partial, hipStream_t stream);

// Per pair of directions: sum the chunk partials, complex FFT of size n,
// multiply by mult (and separately by mult_d when grid_d != nullptr),
// inverse FFT, store the cells [lo, lo+nr) of the real grids.
// LDS bytes of one FFT-convolution workgroup (grid size n, derivative grids)
size_t fftconv_lds_bytes(int n, bool grad);
hipError_t launch_fftconv(const float* partial, int nchunk, int P, GridGeom g,
                          const float2* tw, const float2* mult,
                          const float2* mult_d, float* grid, float* grid_d,
                          hipStream_t stream);

// spart[b*ldm + m] = sum over the directions p of group b (pg per group) of
//   sum_taps grid[p*nr + cell - lo] * window(cell - u(proj[p*ld + m]))
// accumulated in FP64.  If tout != nullptr the per-direction values are
// written to tout[p*ld_t + m] instead and spart is not touched.
hipError_t launch_gather(int W, const float* proj, int64_t ld, int64_t M,
                         int P, GridGeom g, const float* grid, int pg,
                         int pstage, const WindowArgs& win, double* spart,
                         int64_t ldm, float* tout, int64_t ld_t,
                         hipStream_t stream);

// s[m] = (float)(scale * sum_b spart[b*ldm + m]), b < nb; then the bound
// check bc (BoundCheck; bc.norms == nullptr: none).
hipError_t launch_reduce(const double* spart, int nb, int64_t ldm, int64_t M,
                         double scale, float* s, const BoundCheck& bc, hipStream_t stream);

// grad_y[m*d + i] = v[m] * coef * sum_p tprime[p*ld + m] * A[p*dpad + i]
hipError_t launch_backproject(const float* tprime, int64_t ld, int64_t M,
                              int P, int d, const float* A, int dpad,
                              float coef, const float* v, float* grad_y,
                              hipStream_t stream);

// ---- fused projection + spread / gather (d <= kSplitMaxD) ----
//
// Split-f16 operand tiles: a value v (points scaled by 1/R, directions as
// they are) is held as hi = f16(v), lo = f16(v - hi).  Tile t (16 rows),
// k-block kb (32 columns), part q (0 hi, 1 lo) is 1 KB: 64 lanes x 8 halves,
// lane l = c + 16 j holding row 16t + c, columns 32kb + 8j .. +7, zero past
// the rows and columns; byte offset ((t * KB + kb) * 2 + q) * 1024 + 16 l
// with KB = ceil(d / 32).

constexpr int kFuseDirs = 16;        // directions per fused workgroup
constexpr int kSplitMaxD = 64;       // d handled by the fused kernels
constexpr int kSplitTileBytes = 1024;
inline int split_kblocks(int d) { return (d + 31) / 32; }

// true if the fused kernels handle dimension d and grids of nr cells
bool fused_supported(int d, int nr);
// grids too wide for the narrow fused kernels (16 nr > 16384 cells): the
// wide variants (batched plans take only narrow grids)
bool fused_wide(int nr);
// targets per fused gather workgroup (grids of nr cells, window width W)
int64_t fused_gather_tile(int nr, int W);
// resident workgroups per CU of the fused spread and gather kernels
void fused_occupancy(int W, int d, int nr, int* spread_blocks, int* gather_blocks);
// bytes of the split tiles of `rows` rows of dimension d
int64_t split_tiles_bytes(int64_t rows, int d);

// tiles of Z * scale (Z: N x d row-major); sets *flag if a row has
// |Z_row * scale|^2 > norm2_max (or is not finite); records the largest
// |Z_row * scale|^2 in *norm_slot (nullable, see BoundCheck)
hipError_t launch_split_points(const float* Z, int64_t N, int d, float scale, uint16_t* tiles,
                               float norm2_max, int* flag, unsigned* norm_slot,
                               hipStream_t stream);

// As launch_spread, with the projections computed in the kernel from the
// split tiles of the sources (Xt, scale 1/R) and of the directions (At):
// x~ = pscale * <xi, x / R>, pscale = tau R.
hipError_t launch_spread_fused(int W, const uint16_t* Xt, int64_t N, int d, const uint16_t* At,
                               const float* w, int P, GridGeom g, float pscale, int nchunk,
                               int64_t chunk_len, float* slice_max, const WindowArgs& win,
                               float* partial, hipStream_t stream);

// spart[b*ldm + m] = sum over directions p of range b (prange per range, a
// multiple of kFuseDirs) of the interpolated grid at tau <xi_p, y_m>, FP64.
hipError_t launch_gather_fused(int W, const uint16_t* Yt, int64_t M, int d, const uint16_t* At,
                               int P, GridGeom g, float pscale, const float* grid, int prange,
                               const WindowArgs& win, double* spart, int64_t ldm,
                               hipStream_t stream);

// Adjoint in the targets on the fused path:
//   grad_y[m*d + i] = coef * v[m] * sum_p t'_{m,p} (tau xi_p)_i
// with t' the derivative grid interpolated at the in-kernel projections and
// the sum over p back-projected on the matrix cores.  Ab: per 16-direction
// group g, MFMA i (0..3) and 16-coordinate chunk q (DC = ceil(d/16)), 64
// floats: entry k*16 + m = tau xi_{16g + 4k + i}[16q + m] (zero past P, d).
// gpart: ceil(P / prange) x ldg x 16 DC floats of partial sums (ldg >= M).
int64_t fused_grad_tile();    // targets per workgroup
hipError_t launch_grad_fused(int W, const uint16_t* Yt, int64_t M, int d, const uint16_t* At,
                             const float* Ab, int P, GridGeom g, float pscale,
                             const float* grid_d, int prange, const WindowArgs& win,
                             float* gpart, int64_t ldg, float coef, const float* v,
                             float* grad_y, hipStream_t stream);

// ---- exact sliced sums for the energy kernel by sorting (sorted.hip) ----
// Rows of stride L hold, per direction p, the projections of the N sources
// in keys_in[p L + i], i < N, and (same_xy == 0) of the M targets at
// i = yoff + m; entries in [N, yoff) are padding of any value.  Each row's
// first yoff + M (same_xy: N) entries are sorted (keys_out, vals_out =
// original positions p L + i) and each target's per-direction sum
// coef * sum_n w_n |x~_n - y~_m| is computed in FP64 and staged in FP32 by
// 4096-target bucket (stv, with the target's offset in its bucket in sti,
// both P x ldm).  P * L < 2^32.  temp holds sorted_energy_temp_bytes(L, P)
// bytes.  launch_sorted_bucket_reduce then takes the FP64 mean over the
// directions, s[m] = scale * sum_p (per-direction sum), over at most
// kSortMaxRanges direction ranges summed into part (kSortMaxRanges x ldm
// doubles), and finishes with the bound check bc.
constexpr int kSortMaxRanges = 48;
size_t sorted_energy_temp_bytes(int64_t L, int P);
hipError_t launch_sorted_energy(const float* keys_in, float* keys_out, unsigned int* vals_out,
                                void* temp, size_t temp_bytes, int64_t L, int P, int N, int yoff,
                                int M, int same_xy, const float* w, double coef, float* stv,
                                unsigned short* sti, int64_t ldm, hipStream_t stream);
hipError_t launch_sorted_bucket_reduce(const float* stv, const unsigned short* sti, int P,
                                       int64_t ldm, int M, double* part, double scale, float* s,
                                       const BoundCheck& bc, hipStream_t stream);
// s[m] = scale * sum_p V[p ldm + m] (FP64, directions in order), then bc
hipError_t launch_sorted_reduce(const float* V, int P, int64_t ldm, int64_t M, double scale,
                                float* s, const BoundCheck& bc, hipStream_t stream);
// Adjoint pieces per direction from the rows launch_sorted_energy sorted
// (keys_sorted, vals; the same L, N, yoff, M, same_xy; sources at i < N
// with weights w, targets at yoff + m with cotangent v; sign(0) = 0 at
// equal keys), each staged by 4096-index bucket as a P x ldm FP32 value
// row and a P x ldm offset row (as the forward's sums):
//   Ty[p][m] = coef sum_n w_n sign(y~_m - x~_n) (want bit 0; Tyv, Tyo),
//   Tx[p][n] = coef sum_m v_m sign(x~_n - y~_m) (bit 1; Txv, Txo),
//   U[p][n] = coef sum_m v_m |x~_n - y~_m| (bit 2; Uv, Uo).
// launch_sorted_place puts Ty or Tx back in index order (out, P x ldm);
// launch_sorted_bucket_reduce takes the mean of U over the directions.
hipError_t launch_sorted_grad(const float* keys_in, const float* keys_sorted,
                              const unsigned int* vals, int64_t L, int P, int N, int yoff, int M,
                              int same_xy, const float* w, const float* v, double coef,
                              float* Tyv, unsigned short* Tyo, float* Txv, unsigned short* Txo,
                              float* Uv, unsigned short* Uo, int64_t ldm, int want,
                              hipStream_t stream);
hipError_t launch_sorted_place(const float* stv, const unsigned short* sti, int P, int64_t ldm,
                               int M, float* out, hipStream_t stream);

// ---- distance QMC directions (qmc.hip) ----
// iters projected Adam steps on the rows of xi (P x d, d <= 64, unit rows)
// in place; m, v: P x d workspaces; part: distance_qmc_part_floats(P).
size_t distance_qmc_part_floats(int P);
hipError_t distance_qmc(float* xi, int P, int d, int iters, double lr, float* m, float* v,
                        float* part, hipStream_t st);
// Rows of xi (P x d, d <= 64) replaced by Q xi_p / |Q xi_p| (App. E), Q
// device d x d row-major; asynchronous on st.
hipError_t rotate_directions(const float* q, float* xi, int P, int d, hipStream_t st);

// ---- batched form: one persistent launch per phase over a task list ----

// Everything one problem of a batch needs on the device.
struct BatchProblem {
    const float* x;        // N x d sources   (exec time)
    const float* w;        // N weights       (exec time)
    const float* y;        // M x d targets   (exec time)
    float* s;              // M results       (exec time)
    int64_t N, M;
    const float* A;        // tau * Xi^T, P x dpad
    float* xproj;          // P x ldx
    float* yproj;          // P x ldy
    float* partial;        // nchunk x P x nr
    float* grid;           // P x nr
    double* spart;         // ngroup x ldm
    float* slice_max;      // ceil(N / kSliceLen)
    const float2* mult;    // n coefficient multipliers
    const float2* tw;      // n twiddles
    int64_t ldx, ldy, ldm;
    int64_t chunk_len;
    GridGeom g;
    int d, dpad;
    int nchunk, pg, ngroup;      // fused: pg = directions per gather range
    int same_xy;
    float bound;
    // fused problems (d <= kSplitMaxD): split tiles instead of projections
    const uint16_t* at;    // directions, ceil(P/16) tiles
    uint16_t* xt;          // sources, ceil(n_max/16) tiles
    uint16_t* yt;          // targets, ceil(m_max/16) tiles
    float pscale;          // tau R
    float inv_r;           // 1 / R
    float norm2_max;       // range check of |x / R|^2
    int kb;                // ceil(d / 32)
    // bound check (BoundCheck): kNormUints slots of the largest |x / R|^2 of
    // the sources and of the targets, compared with norm_lim by the
    // problem's first reduce task
    unsigned* norms;
    float norm_lim;
};

// One tile of one phase of one problem; a, b, c are phase-specific indices.
struct BatchTask {
    int prob;
    int a;
    int b;
    int c;
};

enum BatchPhase {
    kBatchProject = 0,   // a = 0 (x) / 1 (y), b = point tile, c = direction tile
                         // (fused: b = block of kSplitTaskTiles split tiles)
    kBatchScale = 1,     // a = slice of kSliceLen sources
    kBatchSpread = 2,    // a = direction, b = chunk (fused: a = 16-direction group)
    kBatchFftconv = 3,   // a = direction pair
    kBatchGather = 4,    // a = target tile, b = direction group (fused: range)
    kBatchReduce = 5,    // a = block of kBlock targets
    kBatchPhases = 6
};

constexpr int kSplitTaskTiles = 4;      // split tiles per fused batch task (kBlock / 64)

constexpr int kProjTileP = 64;          // projection tile: directions
constexpr int kProjTileN = 128;         // projection tile: points
constexpr int kGatherTile = 4 * kBlock; // targets per gather tile

hipError_t launch_batch_phase(int phase, int W, const BatchProblem* probs,
                              const BatchTask* tasks, int ntasks, int P, int pstage,
                              const WindowArgs& win, int* flag, int grid_blocks,
                              size_t lds_bytes, hipStream_t stream);
// The split, spread and gather phases of fused batches (every problem with
// d <= kSplitMaxD); the other phases are shared with launch_batch_phase.
// These three run one workgroup per task.
hipError_t launch_batch_phase_fused(int phase, int W, const BatchProblem* probs,
                                    const BatchTask* tasks, int ntasks, int P,
                                    const WindowArgs& win, int* flag, int grid_blocks,
                                    size_t lds_bytes, hipStream_t stream);
// LDS bytes of the fused batch spread / gather workgroups for grids of nr cells
size_t fused_spread_lds(int nr);
// LDS bytes of the stored-projection spread (one direction's int32 cells)
size_t stored_spread_lds(int nr);
size_t fused_gather_lds(int nr);

}  // namespace fastsum
