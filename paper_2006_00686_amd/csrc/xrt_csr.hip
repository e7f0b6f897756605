// The projection matrix in sparse storage: row offsets from per-row counts (exclusive
// scan), a deterministic CSR transpose and a batched CSR product, on gfx950.
//
// A row of A is the hit list of one ray (unit indices and lengths, as xrt_ray_hits
// writes them); its transpose holds, per unit, the rays that hit it.  With A stored, a
// product costs one gather and one multiply-add per nonzero per image instead of the walk
// of every ray, which pays for repeated products on small problems (iterative solves).
#include <hip/hip_runtime.h>

#include "xrt_internal.h"

namespace xrt {
namespace {

constexpr int kSB = 256;            // threads of a scan block
constexpr int kSPer = 4;            // elements per thread
constexpr int kSChunk = kSB * kSPer;

// exclusive scan of one block's kSChunk values (in registers) in LDS; returns the block total
__device__ int64_t block_scan(int64_t (&v)[kSPer], int64_t* s)
{
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kSPer; ++i) {
        const int64_t t = v[i];
        v[i] = sum;
        sum += t;
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums
    for (int d = 1; d < kSB; d <<= 1) {
        const int64_t add = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t before = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
    const int64_t total = s[kSB - 1];
#pragma unroll
    for (int i = 0; i < kSPer; ++i) v[i] += before;
    __syncthreads();
    return total;
}

// phase 1: total of every block of counts
__global__ __launch_bounds__(kSB) void k_scan_sums(const int32_t* __restrict__ counts, int64_t n,
                                                   int64_t* __restrict__ sums)
{
    __shared__ int64_t s[kSB];
    const int64_t base = (int64_t)blockIdx.x * kSChunk + threadIdx.x * kSPer;
    int64_t v[kSPer];
#pragma unroll
    for (int i = 0; i < kSPer; ++i) v[i] = base + i < n ? counts[base + i] : 0;
    const int64_t total = block_scan(v, s);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// phase 2 (one block): exclusive scan of the block totals, in chunks
__global__ __launch_bounds__(kSB) void k_scan_totals(int64_t* __restrict__ sums, int64_t nblocks)
{
    __shared__ int64_t s[kSB];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nblocks; c0 += kSChunk) {
        const int64_t base = c0 + threadIdx.x * kSPer;
        int64_t v[kSPer];
#pragma unroll
        for (int i = 0; i < kSPer; ++i) v[i] = base + i < nblocks ? sums[base + i] : 0;
        const int64_t total = block_scan(v, s);
#pragma unroll
        for (int i = 0; i < kSPer; ++i)
            if (base + i < nblocks) sums[base + i] = v[i] + carry;
        carry += total;
    }
    if (threadIdx.x == 0) sums[nblocks] = carry;
}

// phase 3: offsets[i] = sum of counts[0 .. i), offsets[n] = total
__global__ __launch_bounds__(kSB) void k_scan_apply(const int32_t* __restrict__ counts, int64_t n,
                                                    const int64_t* __restrict__ sums, int64_t nblocks,
                                                    int64_t* __restrict__ offsets)
{
    __shared__ int64_t s[kSB];
    const int64_t base = (int64_t)blockIdx.x * kSChunk + threadIdx.x * kSPer;
    int64_t v[kSPer];
#pragma unroll
    for (int i = 0; i < kSPer; ++i) v[i] = base + i < n ? counts[base + i] : 0;
    block_scan(v, s);
    const int64_t add = sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kSPer; ++i)
        if (base + i < n) offsets[base + i] = v[i] + add;
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[n] = sums[nblocks];
}

__global__ __launch_bounds__(kSB) void k_zero_i32(int32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kSB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSB) p[i] = 0;
}

// nonzeros per column (integer atomics: the totals do not depend on their order);
// entries whose column lies outside [0, n_cols) are dropped here and in k_csr_fill
__global__ __launch_bounds__(kSB) void k_csr_count_cols(const int32_t* __restrict__ col, int64_t nnz, int64_t n_cols,
                                                        int32_t* __restrict__ counts)
{
    for (int64_t e = (int64_t)blockIdx.x * kSB + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kSB) {
        const int32_t c = col[e];
        if (c >= 0 && c < n_cols) atomicAdd(counts + c, 1);
    }
}

// place every nonzero of row r into its column's segment (order within a segment is
// fixed afterwards by k_csr_sort_cols)
__global__ __launch_bounds__(kSB) void k_csr_fill(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                                  const float* __restrict__ val, int64_t n_rows, int64_t n_cols,
                                                  const int64_t* __restrict__ t_off, int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ t_col, float* __restrict__ t_val)
{
    const int64_t r = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (r >= n_rows) return;
    for (int64_t e = off[r]; e < off[r + 1]; ++e) {
        const int32_t c = col[e];
        if (c < 0 || c >= n_cols) continue;
        const int64_t pos = t_off[c] + atomicAdd(cursor + c, 1);
        t_col[pos] = (int32_t)r;
        t_val[pos] = val[e];
    }
}

// sort every column's segment by row (insertion sort; rows are distinct, so the result
// is unique and the transpose deterministic)
__global__ __launch_bounds__(kSB) void k_csr_sort_cols(const int64_t* __restrict__ t_off, int64_t n_cols,
                                                       int32_t* __restrict__ t_col, float* __restrict__ t_val)
{
    const int64_t c = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (c >= n_cols) return;
    const int64_t a = t_off[c], b = t_off[c + 1];
    for (int64_t i = a + 1; i < b; ++i) {
        const int32_t key = t_col[i];
        const float v = t_val[i];
        int64_t j = i - 1;
        while (j >= a && t_col[j] > key) {
            t_col[j + 1] = t_col[j];
            t_val[j + 1] = t_val[j];
            --j;
        }
        t_col[j + 1] = key;
        t_val[j + 1] = v;
    }
}

// y[b][r] = sum_e val[e] x[b][col[e]] over row r, kSpmvBB images per pass: one wavefront
// per row, lanes striding over the row's nonzeros (coalesced index and value loads), FP64
// partial sums reduced across the wavefront in a fixed butterfly order (deterministic).
// The gathers are bounds-checked buffer loads (a column outside the input reads 0).
constexpr int kSpmvBB = 8;
constexpr int kRowsPerBlock = kSB / 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__global__ __launch_bounds__(kSB) void k_csr_spmv(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                                  const float* __restrict__ val, int64_t n_rows, int32_t n_cols,
                                                  int32_t batch, const float* __restrict__ x, float* __restrict__ y)
{
    const int32_t lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= n_rows) return;
    const int32_t b0 = blockIdx.y * kSpmvBB;
    const uint64_t a = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)hi << 32) | lo), (short)0, __builtin_amdgcn_readfirstlane(batch * n_cols * 4), 0x00020000);
    double acc[kSpmvBB];
#pragma unroll
    for (int q = 0; q < kSpmvBB; ++q) acc[q] = 0.0;
    const int64_t e1 = off[r + 1];
    for (int64_t e = off[r] + lane; e < e1; e += 64) {
        const int32_t c = col[e];
        const double v = (double)val[e];
#pragma unroll
        for (int q = 0; q < kSpmvBB; ++q) {
            const int32_t b = b0 + q;
            const int32_t o = (b < batch && c >= 0 && c < n_cols) ? (b * n_cols + c) * 4 : (int32_t)0xFFFFFFF0u;
            acc[q] = fma((double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0)), v,
                         acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < kSpmvBB; ++q) {
        const double t = wave_sum(acc[q]);
        if (lane == 0 && b0 + q < batch) y[(int64_t)(b0 + q) * n_rows + r] = (float)t;
    }
}

// Batch-interleaved product: x_il [n_cols][batch], y_il [n_rows][batch] (batch <= 64).
// One wavefront per row, lane = image: the row's indices and values are wave-uniform
// (scalar loads) and each nonzero gathers the batch's 64 values of one unit from 256
// contiguous bytes.  FP64 accumulation in the row's order.
constexpr int kIlRows = kSB / 64;

__global__ __launch_bounds__(kSB) void k_csr_spmv_il(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                                     const float* __restrict__ val, int64_t n_rows, int32_t n_cols,
                                                     int32_t batch, const float* __restrict__ x_il,
                                                     float* __restrict__ y_il)
{
    const int32_t lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * kIlRows + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= n_rows) return;
    const uint64_t a = (uint64_t)x_il;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)hi << 32) | lo), (short)0, __builtin_amdgcn_readfirstlane(batch * n_cols * 4), 0x00020000);
    const int32_t lane_off = lane < batch ? lane * 4 : (int32_t)0xFFFFFFF0u;
    double acc = 0.0;
    const int64_t e0 = off[r], e1 = off[r + 1];
    // 64 nonzeros at a time: one coalesced load of their indices and values, then each is
    // broadcast from its lane in turn (the gathers of consecutive nonzeros are independent)
    for (int64_t base = e0; base < e1; base += 64) {
        const int64_t e = base + lane;
        const int32_t cl = e < e1 ? col[e] : -1;
        const int32_t vl = e < e1 ? __builtin_bit_cast(int32_t, val[e]) : 0;
        const int32_t cnt = (int32_t)(e1 - base < 64 ? e1 - base : 64);
#pragma unroll 8
        for (int32_t j = 0; j < cnt; ++j) {
            const int32_t c = __builtin_amdgcn_readlane(cl, j);
            const double v = (double)__builtin_bit_cast(float, __builtin_amdgcn_readlane(vl, j));
            const int32_t o = (c >= 0 && c < n_cols) ? c * batch * 4 + lane_off : (int32_t)0xFFFFFFF0u;
            acc = fma((double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0)), v, acc);
        }
    }
    if (lane < batch) y_il[r * batch + lane] = (float)acc;
}

// [batch][n] <-> [n][batch] through an LDS tile of 64 elements x up to 64 images
__global__ __launch_bounds__(kSB) void k_interleave(const float* __restrict__ in, float* __restrict__ out, int64_t n,
                                                    int32_t batch, int32_t to_il)
{
    __shared__ float tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (to_il) {
        for (int32_t b = ty; b < batch; b += kSB / 64)
            if (i0 + tx < n) tile[b][tx] = in[(int64_t)b * n + i0 + tx];
        __syncthreads();
        for (int32_t k = ty; k < 64; k += kSB / 64)
            if (i0 + k < n && tx < batch) out[(i0 + k) * batch + tx] = tile[tx][k];
    } else {
        for (int32_t k = ty; k < 64; k += kSB / 64)
            if (i0 + k < n && tx < batch) tile[tx][k] = in[(i0 + k) * batch + tx];
        __syncthreads();
        for (int32_t b = ty; b < batch; b += kSB / 64)
            if (i0 + tx < n) out[(int64_t)b * n + i0 + tx] = tile[b][tx];
    }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kSB - 1) / kSB); }
unsigned grid_capped(int64_t n) { const int64_t g = (n + kSB - 1) / kSB; return (unsigned)(g < 65536 ? g : 65536); }

xrt_status scan(int64_t n, const int32_t* counts, int64_t* offsets, int64_t* work, hipStream_t s)
{
    const int64_t nblocks = (n + kSChunk - 1) / kSChunk;
    if (nblocks > 0) {
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nblocks), dim3(kSB), 0, s, counts, n, work);
    }
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kSB), 0, s, work, nblocks);
    if (nblocks > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblocks), dim3(kSB), 0, s, counts, n, work, nblocks, offsets);
    else
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kSB), 0, s, counts, n, work, nblocks, offsets);
    return hip_fail(hipGetLastError(), "scan launch");
}

}  // namespace
}  // namespace xrt

using namespace xrt;

extern "C" {

int64_t xrt_scan_workspace(int64_t n)
{
    return n < 0 ? -1 : (n + kSChunk - 1) / kSChunk + 1;
}

xrt_status xrt_offsets_from_counts(int64_t n, const int32_t* d_counts, int64_t* d_offsets, int64_t* d_work,
                                   void* stream)
{
    if (n < 0 || n > ((int64_t)1 << 40) || (n > 0 && !d_counts) || !d_offsets || !d_work) {
        set_error("xrt_offsets_from_counts: bad argument");
        return XRT_E_ARG;
    }
    return scan(n, d_counts, d_offsets, d_work, (hipStream_t)stream);
}

int64_t xrt_csr_transpose_workspace(int64_t n_cols)
{
    return n_cols < 0 ? -1 : 2 * (n_cols + 1) + xrt_scan_workspace(n_cols) + 1;
}

xrt_status xrt_csr_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t* d_off, const int32_t* d_col,
                             const float* d_val, int64_t* d_t_off, int32_t* d_t_col, float* d_t_val, int64_t* d_work,
                             int64_t work_len, void* stream)
{
    if (n_rows < 0 || n_cols < 0 || n_cols > INT32_MAX || n_rows > INT32_MAX || nnz < 0 || !d_off || !d_t_off ||
        !d_work || (nnz > 0 && (!d_col || !d_val || !d_t_col || !d_t_val)) ||
        work_len < xrt_csr_transpose_workspace(n_cols)) {
        set_error("xrt_csr_transpose: bad argument or workspace too small");
        return XRT_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    // workspace: counts / cursor (n_cols int32, in int64 slots) then the scan's block totals
    int32_t* counts = (int32_t*)d_work;
    int64_t* sw = d_work + (n_cols + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_capped(n_cols + 1)), dim3(kSB), 0, s, counts, n_cols + 1);
    if (nnz > 0)
        hipLaunchKernelGGL(k_csr_count_cols, dim3(grid_capped(nnz)), dim3(kSB), 0, s, d_col, nnz, n_cols, counts);
    xrt_status st = scan(n_cols, counts, d_t_off, sw, s);
    if (st != XRT_OK) return st;
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_capped(n_cols + 1)), dim3(kSB), 0, s, counts, n_cols + 1);
    if (n_rows > 0)
        hipLaunchKernelGGL(k_csr_fill, dim3(grid_of(n_rows)), dim3(kSB), 0, s, d_off, d_col, d_val, n_rows, n_cols,
                           d_t_off, counts, d_t_col, d_t_val);
    if (n_cols > 0)
        hipLaunchKernelGGL(k_csr_sort_cols, dim3(grid_of(n_cols)), dim3(kSB), 0, s, d_t_off, n_cols, d_t_col, d_t_val);
    return hip_fail(hipGetLastError(), "xrt_csr_transpose launch");
}

xrt_status xrt_csr_spmv(int64_t n_rows, int64_t n_cols, const int64_t* d_off, const int32_t* d_col, const float* d_val,
                        int32_t batch, const float* d_x, float* d_y, void* stream)
{
    if (n_rows < 0 || n_cols < 0 || batch < 1 || batch > 65535 * kSpmvBB || !d_off || !d_x || !d_y ||
        (int64_t)batch * n_cols * 4 > INT32_MAX - 16 || (n_rows + kRowsPerBlock - 1) / kRowsPerBlock > INT32_MAX) {
        set_error("xrt_csr_spmv: bad argument or input too large for 32-bit offsets");
        return XRT_E_ARG;
    }
    if (n_rows == 0) return XRT_OK;
    const dim3 g((unsigned)((n_rows + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)((batch + kSpmvBB - 1) / kSpmvBB));
    hipLaunchKernelGGL(k_csr_spmv, g, dim3(kSB), 0, (hipStream_t)stream, d_off, d_col, d_val, n_rows, (int32_t)n_cols,
                       batch, d_x, d_y);
    return hip_fail(hipGetLastError(), "xrt_csr_spmv launch");
}

xrt_status xrt_interleave(int64_t n, int32_t batch, int32_t to_interleaved, const float* d_in, float* d_out,
                          void* stream)
{
    if (n < 0 || batch < 1 || batch > 64 || !d_in || !d_out || d_in == d_out) {
        set_error("xrt_interleave: bad argument (batch in [1, 64], distinct buffers)");
        return XRT_E_ARG;
    }
    if (n == 0) return XRT_OK;
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)((n + 63) / 64)), dim3(kSB), 0, (hipStream_t)stream, d_in, d_out, n,
                       batch, to_interleaved ? 1 : 0);
    return hip_fail(hipGetLastError(), "xrt_interleave launch");
}

xrt_status xrt_csr_spmv_interleaved(int64_t n_rows, int64_t n_cols, const int64_t* d_off, const int32_t* d_col,
                                   const float* d_val, int32_t batch, const float* d_x_il, float* d_y_il, void* stream)
{
    if (n_rows < 0 || n_cols < 0 || batch < 1 || batch > 64 || !d_off || !d_x_il || !d_y_il ||
        (int64_t)batch * n_cols * 4 > INT32_MAX - 16 || (n_rows + kIlRows - 1) / kIlRows > INT32_MAX) {
        set_error("xrt_csr_spmv_interleaved: bad argument (batch in [1, 64]) or input too large");
        return XRT_E_ARG;
    }
    if (n_rows == 0) return XRT_OK;
    hipLaunchKernelGGL(k_csr_spmv_il, dim3((unsigned)((n_rows + kIlRows - 1) / kIlRows)), dim3(kSB), 0,
                       (hipStream_t)stream, d_off, d_col, d_val, n_rows, (int32_t)n_cols, batch, d_x_il, d_y_il);
    return hip_fail(hipGetLastError(), "xrt_csr_spmv_interleaved launch");
}

}  // extern "C"
