// Ray-driven kernels of the discrete X-ray transform for gfx950: forward projection,
// scatter adjoint and per-ray hit lists.  The per-ray work (ray construction, clip, slab
// walk with the paper's range condition and length formula) is in xrt_walk.h.
//
// One lane per ray; by default a wavefront holds 64 consecutive rays in (view, row,
// column) order -- 64 neighbouring detector columns of one row -- so neighbouring lanes
// walk neighbouring, nearly parallel rays through the same part of the image (a plan can
// ask for packets of 32 x 2 or 16 x 4 detector cells instead, and an XCD-aware block
// order).  A batch of plans runs as one persistent launch over a queue of ray chunks.
// Image and sinogram data are float32; line integrals accumulate in FP64.
#include <algorithm>

#include "xrt_walk.h"

namespace xrt {
namespace {

constexpr int kBlock = 256;

// Visitors (see walk() for the candidate contract).
//
// Forward: gathers are hardware-bounds-checked buffer loads on byte offsets.  A
// candidate that is not hit is pointed out of range, so its load returns 0 without a
// memory access and its (finite) length adds nothing; the loads of a slab are issued
// together, and the slab's products are summed one slab later, so that the loads'
// latency overlaps the next slab's arithmetic (the order of the sum is unchanged).
constexpr int32_t kOutOfRange = (int32_t)0xFFFFFFF0u;

__device__ __forceinline__ const float* uniform_ptr(const float* p)
{
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (const float*)(((uint64_t)hi << 32) | lo);
}

// Buffer resource of a wave-uniform image (base and size taken from the first lane).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const float* img, int32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)uniform_ptr(img), (short)0, __builtin_amdgcn_readfirstlane(nbytes),
                                             0x00020000);
}

struct FwdVisit {
    static constexpr int32_t kIndexScale = 4;
    __amdgpu_buffer_rsrc_t rsrc;   // the image (built once per ray, outside the walk)
    double acc;
    // the previous slab's loaded values and lengths, consumed after this slab's loads
    // are issued (their latency overlaps the next slab's arithmetic)
    float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    double q1 = 0.0, q2 = 0.0, q3 = 0.0;
    __device__ __forceinline__ float load(int32_t off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
    }
    __device__ __forceinline__ void consume()
    {
        acc = fma((double)p1, q1, acc);
        acc = fma((double)p2, q2, acc);
        acc = fma((double)p3, q3, acc);
    }
    // h2, h3: the walk's flags (the candidate may have a positive length); a candidate
    // that cannot reads out of range (0).  In 3D the second candidate's load keeps its
    // length test: issued after the lengths, the loads leave the previous slab's values
    // time to arrive before they are summed (256^3 cone forward: both length tests
    // 11.28 ms, both flags 11.49 ms -- the loads moved ahead and the sums waited --, this
    // mix 11.06 ms)
    __device__ __forceinline__ void two_h(int32_t I1, double l1, int32_t I2, double l2, bool h2)
    {
        const float f1 = load(I1);
        const float f2 = load(h2 ? I2 : kOutOfRange);
        consume();
        p1 = f1;
        p2 = f2;
        p3 = 0.0f;
        q1 = l1;
        q2 = l2;
        q3 = 0.0;
    }
    __device__ __forceinline__ void three_h(int32_t I1, double l1, int32_t I2, double l2, bool h2, int32_t I3,
                                            double l3, bool h3)
    {
        const float f1 = load(I1);
        const float f2 = load(l2 > 0.0 ? I2 : kOutOfRange);
        const float f3 = load(h3 ? I3 : kOutOfRange);
        consume();
        p1 = f1;
        p2 = f2;
        p3 = f3;
        q1 = l1;
        q2 = l2;
        q3 = l3;
    }
};

// FwdVisit for 2D walks, whose slabs have two candidates: the loaded values are summed
// two slabs after their loads are issued (same order of the sum), so that up to four
// loads of a lane are in flight.
struct FwdVisit2 {
    static constexpr int32_t kIndexScale = 4;
    __amdgpu_buffer_rsrc_t rsrc;
    double acc;
    float p1 = 0.0f, p2 = 0.0f, r1 = 0.0f, r2 = 0.0f;     // two slabs ago, one slab ago
    double q1 = 0.0, q2 = 0.0, s1 = 0.0, s2 = 0.0;
    __device__ __forceinline__ float load(int32_t off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
    }
    __device__ __forceinline__ void consume()
    {
        acc = fma((double)p1, q1, acc);
        acc = fma((double)p2, q2, acc);
        acc = fma((double)r1, s1, acc);
        acc = fma((double)r2, s2, acc);
    }
    __device__ __forceinline__ void two_h(int32_t I1, double l1, int32_t I2, double l2, bool h2)
    {
        const float f1 = load(I1);
        const float f2 = load(h2 ? I2 : kOutOfRange);
        acc = fma((double)p1, q1, acc);
        acc = fma((double)p2, q2, acc);
        p1 = r1;
        p2 = r2;
        q1 = s1;
        q2 = s2;
        r1 = f1;
        r2 = f2;
        s1 = l1;
        s2 = l2;
    }
    __device__ __forceinline__ void three_h(int32_t, double, int32_t, double, bool, int32_t, double, bool) {}
};

// FwdVisit for a batch in the lanes of a wavefront: every lane walks the same ray (the
// walk's values are the same in all lanes) and reads its own image's value of each unit
// from the interleaved layout [unit][image], so the batch's values of a unit are one
// contiguous load.  off(I) = I * 4 batch + 4 lane.
struct FwdBatchVisit {
    static constexpr int32_t kIndexScale = 1;
    __amdgpu_buffer_rsrc_t rsrc;
    int32_t stride4, lane4;
    double acc;
    float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    double q1 = 0.0, q2 = 0.0, q3 = 0.0;
    __device__ __forceinline__ float load(bool hit, int32_t I)
    {
        return __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, hit ? I * stride4 + lane4 : kOutOfRange, 0, 0));
    }
    __device__ __forceinline__ void consume()
    {
        acc = fma((double)p1, q1, acc);
        acc = fma((double)p2, q2, acc);
        acc = fma((double)p3, q3, acc);
    }
    __device__ __forceinline__ void two_h(int32_t I1, double l1, int32_t I2, double l2, bool h2)
    {
        const float f1 = load(true, I1);
        const float f2 = load(h2, I2);
        consume();
        p1 = f1;
        p2 = f2;
        p3 = 0.0f;
        q1 = l1;
        q2 = l2;
        q3 = 0.0;
    }
    __device__ __forceinline__ void three_h(int32_t I1, double l1, int32_t I2, double l2, bool h2, int32_t I3,
                                            double l3, bool h3)
    {
        const float f1 = load(true, I1);
        const float f2 = load(h2, I2);
        const float f3 = load(h3, I3);
        consume();
        p1 = f1;
        p2 = f2;
        p3 = f3;
        q1 = l1;
        q2 = l2;
        q3 = l3;
    }
};

// img[I] += val for the lanes with hit, where neighbouring lanes -- neighbouring detector
// columns, which often cross the same unit in a slab -- that add to one unit do so with
// one atomic: each run of consecutive lanes with the same I adds its sum from its first
// lane (256^3 cone attenuated adjoint 141 -> 95 ms: the atomics cost per lane).  Every
// lane of the wavefront that reaches the call takes part; lanes without a hit pass
// hit = false and add nothing.
__device__ __forceinline__ void atomic_add_runs(float* img, int32_t I, bool hit, float val)
{
    const uint32_t lane = __lane_id();
    const uint64_t act = __builtin_amdgcn_ballot_w64(true);
    const int32_t key = hit ? I : -1;
    const int32_t kn = __shfl_down(key, 1);
    const bool nxt = lane < 63 && ((act >> (lane + 1)) & 1ull);
    const uint64_t cont = __builtin_amdgcn_ballot_w64(hit && nxt && kn == key);   // lane + 1 in my run
    float acc = val, v = val;
    // pass d adds the value of lane + d to the lanes whose run reaches that far
    for (uint64_t run = cont, d = 1; run != 0; run &= cont >> d, ++d) {
        v = __shfl_down(v, 1);
        if ((run >> lane) & 1ull) acc += v;
    }
    if (hit && !(lane > 0 && ((cont >> (lane - 1)) & 1ull))) unsafeAtomicAdd(img + I, acc);
}

// Before the runs merge: a lane's second unit of a slab is often the first unit of a
// neighbouring lane (the neighbouring ray is already past the boundary this one crosses).
// Such a value is handed to that lane, whose first-unit run then adds it, and the lane
// keeps no atomic for it (keep2 = false).  A value goes to the lane above (lane + 1) if
// that lane takes it, else to the lane below if that one does -- never to both.
__device__ __forceinline__ void hand_over(int32_t I1, bool hit1, float& v1, int32_t I2, bool hit2, float v2,
                                          bool& keep2)
{
    const uint32_t lane = __lane_id();
    const uint64_t act = __builtin_amdgcn_ballot_w64(true);
    const int32_t k2 = hit2 ? I2 : -2;
    const int32_t kb = __shfl_up(k2, 1), ka = __shfl_down(k2, 1);
    const float vb = __shfl_up(v2, 1), va = __shfl_down(v2, 1);
    const bool has_b = lane > 0 && ((act >> (lane - 1)) & 1ull);
    const bool has_a = lane < 63 && ((act >> (lane + 1)) & 1ull);
    const bool tb = hit1 && has_b && kb == I1;                      // from the lane below
    const uint64_t TB = __builtin_amdgcn_ballot_w64(tb);
    const bool ta = hit1 && has_a && ka == I1 && !(lane + 2 < 64 && ((TB >> (lane + 2)) & 1ull));
    const uint64_t TA = __builtin_amdgcn_ballot_w64(ta);
    if (tb) v1 += vb;
    if (ta) v1 += va;
    keep2 = hit2 && !((lane < 63 && ((TB >> (lane + 1)) & 1ull)) || (lane > 0 && ((TA >> (lane - 1)) & 1ull)));
}

struct ScatterVisit {
    static constexpr int32_t kIndexScale = 1;
    float* img;
    double gw;
    __device__ __forceinline__ void one(int32_t I, double l)
    {
        atomic_add_runs(img, I, l > 0.0, (float)(gw * l));
    }
    __device__ __forceinline__ void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        float v1 = (float)(gw * l1);
        bool keep2;
        hand_over(I1, l1 > 0.0, v1, I2, l2 > 0.0, (float)(gw * l2), keep2);
        atomic_add_runs(img, I1, l1 > 0.0, v1);
        atomic_add_runs(img, I2, keep2, (float)(gw * l2));
    }
    __device__ __forceinline__ void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3,
                                          double l3)
    {
        float v1 = (float)(gw * l1);
        bool keep2;
        hand_over(I1, l1 > 0.0, v1, I2, l2 > 0.0, (float)(gw * l2), keep2);
        atomic_add_runs(img, I1, l1 > 0.0, v1);
        atomic_add_runs(img, I2, keep2, (float)(gw * l2));
        one(I3, l3);
    }
};

struct CountVisit {
    static constexpr int32_t kIndexScale = 1;
    double thr;     // eps / scale
    int32_t n;
    __device__ __forceinline__ void two(int32_t, double l1, int32_t, double l2)
    {
        n += (l1 > thr) + (l2 > thr);
    }
    __device__ __forceinline__ void three(int32_t, double l1, int32_t, double l2, int32_t, double l3)
    {
        n += (l1 > thr) + (l2 > thr) + (l3 > thr);
    }
};

struct EmitVisit {
    static constexpr int32_t kIndexScale = 1;
    int32_t* idx;
    float* len;
    double thr, scale;
    int32_t n, cap;
    __device__ __forceinline__ void one(int32_t I, double l)
    {
        if (l > thr && n < cap) {
            idx[n] = I;
            len[n] = (float)(l * scale);
            ++n;
        }
    }
    __device__ __forceinline__ void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        one(I1, l1);
        one(I2, l2);
    }
    __device__ __forceinline__ void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3,
                                          double l3)
    {
        one(I1, l1);
        one(I2, l2);
        one(I3, l3);
    }
};

// Attenuated transform (the generalised transform of the paper's Introduction with the
// SPECT weight exp(-integral of mu from the point to the detector side of the ray)).  The
// walk runs from the detector side back (the ray's direction reversed), so for every piece
// the attenuation between it and the detector is the running sum A of mu * length over
// the pieces already visited; a piece of length len with values f, mu contributes
// f exp(-A) (1 - exp(-mu len)) / mu  (f len when mu = 0), its exact integral.
// Weight (1 - exp(-x)) / mu of a piece, x = mu * len, in FP32: for |x| < 0.05 by its
// series len (1 - x/2 + x^2/6 - x^3/24) (truncation < 6e-8 relative, no cancellation),
// above it directly (relative error ~1e-6 at x = 0.05, less beyond).
__device__ __forceinline__ float att_weight(float m, float lp, float x)
{
    if (fabsf(x) < 0.05f) return lp * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f))));
    return (1.0f - __expf(-x)) / m;
}

struct AttFwdVisit {
    static constexpr int32_t kIndexScale = 4;
    __amdgpu_buffer_rsrc_t rf, rm;   // image and attenuation map
    double scale;                     // physical length per unit of ray parameter
    double A;                         // attenuation between the current piece and the detector
    double acc;
    // the previous slab's values and lengths, processed (in order) after this slab's
    // loads are issued, as in the plain forward
    float pf[3] = {0.0f, 0.0f, 0.0f}, pm[3] = {0.0f, 0.0f, 0.0f};
    double pl[3] = {0.0, 0.0, 0.0};
    __device__ __forceinline__ float ld(const __amdgpu_buffer_rsrc_t& r, int32_t off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    // one piece: a candidate that is not hit has f = mu = 0 (out of range) and length
    // <= 0 (clamped to 0, so that the FP32 weight stays finite): it adds nothing.  A is
    // summed in FP64; exp(-A) and the weight are FP32 (relative error ~1e-6 with A up to
    // ~20, far below the transform's tolerance)
    __device__ __forceinline__ void piece(float f, float m, double l)
    {
        const double lp = fmax(l, 0.0) * scale, x = (double)m * lp;
        const float w = att_weight(m, (float)lp, (float)x);
        acc = fma((double)(f * __expf(-(float)A)), (double)w, acc);
        A += x;
    }
    __device__ __forceinline__ void consume()
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) piece(pf[i], pm[i], pl[i]);
    }
    __device__ __forceinline__ void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        const int32_t o2 = l2 > 0.0 ? I2 : kOutOfRange;
        const float f1 = ld(rf, I1), m1 = ld(rm, I1), f2 = ld(rf, o2), m2 = ld(rm, o2);
        consume();
        pf[0] = f1;
        pm[0] = m1;
        pl[0] = l1;
        pf[1] = f2;
        pm[1] = m2;
        pl[1] = l2;
        pf[2] = 0.0f;
        pm[2] = 0.0f;
        pl[2] = 0.0;
    }
    __device__ __forceinline__ void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3,
                                          double l3)
    {
        const int32_t o2 = l2 > 0.0 ? I2 : kOutOfRange, o3 = l3 > 0.0 ? I3 : kOutOfRange;
        const float f1 = ld(rf, I1), m1 = ld(rm, I1), f2 = ld(rf, o2), m2 = ld(rm, o2), f3 = ld(rf, o3),
                    m3 = ld(rm, o3);
        consume();
        pf[0] = f1;
        pm[0] = m1;
        pl[0] = l1;
        pf[1] = f2;
        pm[1] = m2;
        pl[1] = l2;
        pf[2] = f3;
        pm[2] = m3;
        pl[2] = l3;
    }
};

// AttFwdVisit reading (f, mu) pairs: one 8-byte load per candidate.
struct AttFwdPairVisit {
    static constexpr int32_t kIndexScale = 8;
    __amdgpu_buffer_rsrc_t rp;   // (f, mu) pairs
    double scale, A, acc;
    float pf[3] = {0.0f, 0.0f, 0.0f}, pm[3] = {0.0f, 0.0f, 0.0f};
    double pl[3] = {0.0, 0.0, 0.0};
    __device__ __forceinline__ void ld(int32_t off, float& f, float& m)
    {
        f = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, off, 0, 0));
        m = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, off + 4, 0, 0));
    }
    // as AttFwdVisit::piece
    __device__ __forceinline__ void piece(float f, float m, double l)
    {
        const double lp = fmax(l, 0.0) * scale, x = (double)m * lp;
        const float w = att_weight(m, (float)lp, (float)x);
        acc = fma((double)(f * __expf(-(float)A)), (double)w, acc);
        A += x;
    }
    __device__ __forceinline__ void consume()
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) piece(pf[i], pm[i], pl[i]);
    }
    __device__ __forceinline__ void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        float f1, m1, f2, m2;
        ld(I1, f1, m1);
        ld(l2 > 0.0 ? I2 : kOutOfRange, f2, m2);
        consume();
        pf[0] = f1;
        pm[0] = m1;
        pl[0] = l1;
        pf[1] = f2;
        pm[1] = m2;
        pl[1] = l2;
        pf[2] = 0.0f;
        pm[2] = 0.0f;
        pl[2] = 0.0;
    }
    __device__ __forceinline__ void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3,
                                          double l3)
    {
        float f1, m1, f2, m2, f3, m3;
        ld(I1, f1, m1);
        ld(l2 > 0.0 ? I2 : kOutOfRange, f2, m2);
        ld(l3 > 0.0 ? I3 : kOutOfRange, f3, m3);
        consume();
        pf[0] = f1;
        pm[0] = m1;
        pl[0] = l1;
        pf[1] = f2;
        pm[1] = m2;
        pl[1] = l2;
        pf[2] = f3;
        pm[2] = m3;
        pl[2] = l3;
    }
};

struct AttAdjVisit {
    static constexpr int32_t kIndexScale = 1;
    float* img;
    __amdgpu_buffer_rsrc_t rm;
    double scale, g, A;
    // the piece's value g exp(-A) w, A then taking the piece (0 for a candidate not hit)
    __device__ __forceinline__ float value(int32_t I, double l)
    {
        float val = 0.0f;
        if (l > 0.0) {
            const float m = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rm, I * 4, 0, 0));
            const double lp = l * scale, x = (double)m * lp;
            const float w = att_weight(m, (float)lp, (float)x);
            val = (float)(g * (double)(__expf(-(float)A) * w));
            A += x;
        }
        return val;
    }
    __device__ __forceinline__ void one(int32_t I, double l)
    {
        const float val = value(I, l);
        atomic_add_runs(img, I, l > 0.0, val);
    }
    __device__ __forceinline__ void two(int32_t I1, double l1, int32_t I2, double l2)
    {
        float v1 = value(I1, l1);
        const float v2 = value(I2, l2);
        bool keep2;
        hand_over(I1, l1 > 0.0, v1, I2, l2 > 0.0, v2, keep2);
        atomic_add_runs(img, I1, l1 > 0.0, v1);
        atomic_add_runs(img, I2, keep2, v2);
    }
    __device__ __forceinline__ void three(int32_t I1, double l1, int32_t I2, double l2, int32_t I3,
                                          double l3)
    {
        float v1 = value(I1, l1);
        const float v2 = value(I2, l2);
        bool keep2;
        hand_over(I1, l1 > 0.0, v1, I2, l2 > 0.0, v2, keep2);
        atomic_add_runs(img, I1, l1 > 0.0, v1);
        atomic_add_runs(img, I2, keep2, v2);
        one(I3, l3);
    }
};

// Ray of thread t when a wavefront covers a packet of P.packet_cols detector columns x
// (64 / packet_cols) rows of one view, or -1 past the detector's edge.
__device__ __forceinline__ int32_t packet_ray(const DevPlan& P, uint64_t t)
{
    const uint32_t tw = (uint32_t)P.packet_cols, th = 64u / tw;
    const uint32_t ct = ((uint32_t)P.n_cols + tw - 1) / tw, rt = ((uint32_t)P.n_rows + th - 1) / th;
    const uint64_t packet = t >> 6, per_view = (uint64_t)ct * rt;
    const uint32_t lane = (uint32_t)t & 63u;
    const uint64_t view = packet / per_view;
    if (view >= (uint64_t)P.n_views) return -1;
    const uint32_t rem = (uint32_t)(packet - view * per_view);
    const uint32_t rti = rem / ct, cti = rem - rti * ct;
    const uint32_t row = rti * th + lane / tw, col = cti * tw + lane % tw;
    if (row >= (uint32_t)P.n_rows || col >= (uint32_t)P.n_cols) return -1;
    return (int32_t)(((uint32_t)view * (uint32_t)P.n_rows + row) * (uint32_t)P.n_cols + col);
}

// Ray of thread t of a forward launch (-1: no ray).
template <int MODE>
__device__ __forceinline__ int32_t forward_ray_of(const DevPlan& P, uint64_t t)
{
    if (MODE != MODE_LIST && P.packet_cols > 0) return packet_ray(P, t);
    return t < (uint64_t)P.n_rays ? (int32_t)t : -1;
}

// Threads a forward launch enumerates.
__host__ __device__ inline uint64_t forward_threads(const DevPlan& P)
{
    if (P.mode == MODE_LIST || P.packet_cols == 0) return (uint64_t)P.n_rays;
    const uint64_t tw = (uint64_t)P.packet_cols, th = 64u / tw;
    return (uint64_t)P.n_views * ((P.n_cols + tw - 1) / tw) * ((P.n_rows + th - 1) / th) * 64u;
}

// A wavefront's rays step along the image with its lanes spread along the detector's u
// axis; where u runs closer to y than to x, a scatter into the y-fastest layout keeps a
// wavefront's atomic adds in few cache lines (the view's choice, as the forward's).
template <int MODE>
__device__ __forceinline__ bool view_prefers_y_fastest(const DevPlan& P, int32_t r)
{
    if constexpr (MODE == MODE_LIST) {
        return false;
    } else {
        const uint32_t per_view = (uint32_t)P.n_rows * (uint32_t)P.n_cols;
        const uint32_t view0 = __builtin_amdgcn_readfirstlane((uint32_t)r / per_view);
        const ViewGeom& V = P.views[view0];
        return fabs(V.B[1]) > fabs(V.B[0]);
    }
}

// Whether this lane's rays would rather read the y-fastest copy: the lanes of a
// wavefront walk neighbouring rays one slab per step, so at every step they sit where
// their entry points sit, shifted along the ray -- spread along the entry face.  A chord
// entering through an x face (x = const) spreads the lanes along y, one entering
// through a y face along x, one entering through a z face along the detector's u axis.
// The layout whose fastest axis is that spread keeps the wavefront's gathers in few cache
// lines.
template <int DIM>
__device__ __forceinline__ bool prefers_y_fastest(const DevPlan& P, const Ray& R, double bx, double by)
{
    const int32_t n[3] = {P.nx, P.ny, P.nz};
    double best = -kInf;
    int entry = -1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (R.w[a] != 0.0) {
            const double inv = 1.0 / R.w[a];
            const double t = fmin((0.0 - R.q[a]) * inv, ((double)n[a] - R.q[a]) * inv);
            if (t > best) {
                best = t;
                entry = a;
            }
        }
    }
    if (entry == 0) return true;
    if (entry == 1) return false;
    return fabs(by) > fabs(bx);
}

// One ray of the forward projection.  imgT: the same image with y fastest ([z][x][y]),
// or NULL.  In 2D a wavefront reads it when most of its lanes' chords enter the image
// through a face that spreads them along y (prefers_y_fastest; a vote, so the whole
// wavefront reads one layout; fan2d_512 forward 0.352 -> 0.316 ms).  In 3D every
// wavefront of a view reads one layout, the y-fastest copy when the detector's u axis
// runs closer to y than to x: choosing per wavefront there made the waves of a view read
// both copies of the volume, whose L2 working set then doubled (256^3 cone forward
// 18.9 -> 20.8 ms).
// imgZ: the image with z fastest ([y][x][z]) for column packets (packet_cols = 1), whose
// lanes share their xy path and differ in z only, or NULL.
template <int DIM, int MODE, bool NEST = false>
__device__ __forceinline__ void forward_one(const DevPlan& P, int32_t r, const float* img, const float* imgT,
                                            float* sino, const float* wt = nullptr, const float* imgZ = nullptr)
{
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
    const float* base = img;
    if constexpr (MODE != MODE_LIST && DIM == 3) {
        if (imgZ != nullptr) {
            base = imgZ;
            R.st[0] = P.nz;
            R.st[1] = P.nx * P.nz;
            R.st[2] = 1;
            imgT = nullptr;
        }
    }
    if constexpr (MODE != MODE_LIST) {
        if (imgT != nullptr) {
            const uint32_t per_view = (uint32_t)P.n_rows * (uint32_t)P.n_cols;
            const uint32_t view0 = __builtin_amdgcn_readfirstlane((uint32_t)r / per_view);
            const ViewGeom& V = P.views[view0];
            bool use_t = fabs(V.B[1]) > fabs(V.B[0]);
            if constexpr (DIM == 2) {
                const uint64_t want = __builtin_amdgcn_ballot_w64(prefers_y_fastest<DIM>(P, R, V.B[0], V.B[1]));
                const uint64_t all = __builtin_amdgcn_ballot_w64(true);
                use_t = 2 * __builtin_popcountll(want) > __builtin_popcountll(all);
            }
            if (use_t) {
                base = imgT;
                R.st[0] = P.ny;
                R.st[1] = 1;
            }
        }
    }
    std::conditional_t<DIM == 2, FwdVisit2, FwdVisit> v{image_rsrc(base, (int32_t)(P.n_units * 4)), 0.0};
    walk<DIM, NEST>(P, R, v);
    v.consume();
    // wt: a per-ray weight (the PET form of the generalised transform), or none
    const double w = wt != nullptr ? (double)wt[r] : 1.0;
    sino[r] = (float)(v.acc * R.scale * w);
}

// nblocks: workgroups that carry rays; with xcd_remap the grid is rounded up to a
// multiple of 8 and workgroup b takes logical block (b % 8) * (grid / 8) + b / 8.
template <int DIM, int MODE, bool NEST>
__global__ __launch_bounds__(kBlock) void k_forward(DevPlan P, const float* __restrict__ img,
                                                     const float* __restrict__ imgT, float* __restrict__ sino,
                                                     uint32_t nblocks, const float* __restrict__ wt,
                                                     int64_t wt_stride, const float* __restrict__ imgZ)
{
    uint32_t blk = blockIdx.x;
    if (P.xcd_remap) {
        blk = (blk & 7u) * (gridDim.x >> 3) + (blk >> 3);
        if (blk >= nblocks) return;
    }
    const int32_t r = forward_ray_of<MODE>(P, (uint64_t)blk * kBlock + threadIdx.x);
    if (r < 0) return;
    const int64_t b = blockIdx.y;
    forward_one<DIM, MODE, NEST>(P, r, img + b * P.n_units, imgT, sino + b * P.n_rays,
                           wt != nullptr ? wt + b * wt_stride : nullptr, imgZ);
}

// ------------------------------------------------------------------ batched (several plans)
// One persistent launch projects every member of a batch.  The work queue lists chunks
// of kChunkBlocks x 256 threads member by member, members in the order the host chose
// (longest rays first); each workgroup takes the next chunk from a counter until the
// queue is exhausted, so a workgroup that drew short rays simply takes more chunks.
constexpr int kChunkBlocks = 16;

struct BatchQueue {
    int32_t n;                              // members
    int32_t member[kMaxBatch];              // member of queue slot s
    int64_t first_chunk[kMaxBatch + 1];     // first chunk of slot s; [n] = total
    int64_t nblocks[kMaxBatch];             // 256-thread blocks of slot s
};

struct BatchIO {
    const float* in[kMaxBatch];
    const float* inT[kMaxBatch];
    const float* inZ[kMaxBatch];   // z-fastest copy for members with column packets, or NULL
    float* out[kMaxBatch];
};

template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_forward_batch(const DevPlan* __restrict__ plans, BatchQueue q, BatchIO io,
                                                           unsigned long long* __restrict__ counter)
{
    __shared__ unsigned long long s_chunk;
    const int64_t total = q.first_chunk[q.n];
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t chunk = (int64_t)s_chunk;
        __syncthreads();
        if (chunk >= total) break;
        int32_t s = 0;
        while (s + 1 < q.n && chunk >= q.first_chunk[s + 1]) ++s;
        const int32_t m = q.member[s];
        const DevPlan& P = plans[m];
        const int64_t blk0 = (chunk - q.first_chunk[s]) * kChunkBlocks;
        for (int c = 0; c < kChunkBlocks; ++c) {
            const int64_t blk = blk0 + c;
            if (blk >= q.nblocks[s]) break;
            const int32_t r = forward_ray_of<MODE>(P, (uint64_t)blk * kBlock + threadIdx.x);
            if (r >= 0) forward_one<DIM, MODE>(P, r, io.in[m], io.inT[m], io.out[m], nullptr, io.inZ[m]);
        }
    }
}

// mu_stride: 0 (one attenuation map for every image) or the image size
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_forward_att(DevPlan P, const float* __restrict__ img,
                                                         const float* __restrict__ mu, int64_t mu_stride,
                                                         float* __restrict__ sino)
{
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.n_rays) return;
    const int64_t b = blockIdx.y;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
#pragma unroll
    for (int a = 0; a < 3; ++a) R.w[a] = -R.w[a];   // from the detector side back
    const int32_t nb = (int32_t)(P.n_units * 4);
    AttFwdVisit v{image_rsrc(img + b * P.n_units, nb), image_rsrc(mu + b * mu_stride, nb), R.scale, 0.0, 0.0};
    walk<DIM>(P, R, v);
    v.consume();
    sino[b * P.n_rays + r] = (float)v.acc;
}

// Forward projection of a batch of up to 64 images held interleaved ([unit][image]):
// one wavefront per ray, lane = image.  Each (ray, image) takes the same arithmetic in
// the same order as k_forward.  Lanes past the batch repeat an image and store nothing.
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_forward_il(DevPlan P, const float* __restrict__ img,
                                                        float* __restrict__ sino, int32_t batch)
{
    const int32_t r = (int32_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (r >= P.n_rays) return;
    const int32_t lane = threadIdx.x & 63;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
    FwdBatchVisit v{image_rsrc(img, (int32_t)(P.n_units * batch * 4)), 4 * batch, 4 * (lane % batch), 0.0};
    walk<DIM>(P, R, v);
    v.consume();
    if (lane < batch) sino[(int64_t)r * batch + lane] = (float)(v.acc * R.scale);
}

// The attenuated forward of one image from its (f, mu) pairs (NEST: the walk's form).
// ZP: column packets (packet_cols = 1, 64 rows of one detector column per wavefront,
// flat walk) over pairs held z fastest ([y][x][z]), as the plain forward's column packets.
template <int DIM, int MODE, bool NEST, bool ZP = false>
__global__ __launch_bounds__(kBlock) void k_forward_att_pairs(DevPlan P, const float* __restrict__ pairs,
                                                               float* __restrict__ sino)
{
    int32_t r;
    if constexpr (ZP) {
        r = packet_ray(P, (uint64_t)blockIdx.x * kBlock + threadIdx.x);
        if (r < 0) return;
    } else {
        r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
        if (r >= P.n_rays) return;
    }
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
#pragma unroll
    for (int a = 0; a < 3; ++a) R.w[a] = -R.w[a];   // from the detector side back
    if constexpr (ZP) {
        R.st[0] = P.nz;
        R.st[1] = P.nx * P.nz;
        R.st[2] = 1;
    }
    AttFwdPairVisit v{image_rsrc(pairs, (int32_t)(P.n_units * 8)), R.scale, 0.0, 0.0};
    walk<DIM, NEST>(P, R, v);
    v.consume();
    sino[r] = (float)v.acc;
}

// pairs[y][x][z] = (img[z][y][x], mu[z][y][x]) (one y per block row of tiles: 32 z x 32 x)
__global__ __launch_bounds__(kBlock) void k_att_pairs_zfast(const float* __restrict__ img, const float* __restrict__ mu,
                                                             float2* __restrict__ out, int32_t nx, int32_t ny,
                                                             int32_t nz, int32_t ztiles)
{
    __shared__ float2 tile[32][33];
    const int32_t y = blockIdx.y / ztiles;
    const int32_t z0 = (blockIdx.y - y * ztiles) * 32, x0 = blockIdx.x * 32;
    const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int32_t zz = ty; zz < 32; zz += kBlock / 32) {
        const int32_t z = z0 + zz, x = x0 + tx;
        if (z < nz && x < nx) {
            const int64_t at = ((int64_t)z * ny + y) * nx + x;
            tile[zz][tx] = make_float2(img[at], mu[at]);
        }
    }
    __syncthreads();
    for (int32_t xx = ty; xx < 32; xx += kBlock / 32) {
        const int32_t x = x0 + xx, z = z0 + tx;
        if (z < nz && x < nx) out[((int64_t)y * nx + x) * nz + z] = tile[tx][xx];
    }
}

// pairs[i] = (img[i], mu[i])
__global__ __launch_bounds__(kBlock) void k_att_pairs(const float* __restrict__ img, const float* __restrict__ mu,
                                                       float2* __restrict__ pairs, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        pairs[i] = make_float2(img[i], mu[i]);
}

template <int DIM, int MODE>
// imgT, muT (one image, y fastest; imgT zeroed) or NULL: views whose u axis runs along y
// read the map from muT and add into imgT (see view_prefers_y_fastest).
__global__ __launch_bounds__(kBlock) void k_adjoint_att(DevPlan P, const float* __restrict__ sino,
                                                         const float* __restrict__ mu, int64_t mu_stride, float* img,
                                                         float* imgT, const float* __restrict__ muT)
{
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.n_rays) return;
    const int64_t b = blockIdx.y;
    const float g = sino[b * P.n_rays + r];
    if (g == 0.0f) return;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
#pragma unroll
    for (int a = 0; a < 3; ++a) R.w[a] = -R.w[a];
    float* out = img + b * P.n_units;
    const float* m = mu + b * mu_stride;
    if (imgT != nullptr && view_prefers_y_fastest<MODE>(P, r)) {
        out = imgT;
        m = muT;
        R.st[0] = P.ny;
        R.st[1] = 1;
    }
    AttAdjVisit v{out, image_rsrc(m, (int32_t)(P.n_units * 4)), R.scale, (double)g, 0.0};
    walk<DIM>(P, R, v);
}

__global__ void k_reset_counter(unsigned long long* c)
{
    if (threadIdx.x == 0) *c = 0ull;
}

// out[z][x][y] = in[z][y][x]
__global__ __launch_bounds__(kBlock) void k_transpose_xy(const float* __restrict__ in, float* __restrict__ out,
                                                          int32_t nx, int32_t ny, int32_t ytiles)
{
    __shared__ float tile[32][33];
    const int32_t z = blockIdx.y / ytiles;
    const int32_t y0 = (blockIdx.y - z * ytiles) * 32, x0 = blockIdx.x * 32;
    const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t slab = (int64_t)z * nx * ny;
    for (int32_t yy = ty; yy < 32; yy += kBlock / 32) {
        const int32_t y = y0 + yy, x = x0 + tx;
        if (y < ny && x < nx) tile[yy][tx] = in[slab + (int64_t)y * nx + x];
    }
    __syncthreads();
    for (int32_t xx = ty; xx < 32; xx += kBlock / 32) {
        const int32_t x = x0 + xx, y = y0 + tx;
        if (y < ny && x < nx) out[slab + (int64_t)x * ny + y] = tile[tx][xx];
    }
}

// out[y][x][z] = in[z][y][x] (one y per block row of tiles: 32 z x 32 x)
__global__ __launch_bounds__(kBlock) void k_transpose_zfast(const float* __restrict__ in, float* __restrict__ out,
                                                             int32_t nx, int32_t ny, int32_t nz, int32_t ztiles)
{
    __shared__ float tile[32][33];
    const int32_t y = blockIdx.y / ztiles;
    const int32_t z0 = (blockIdx.y - y * ztiles) * 32, x0 = blockIdx.x * 32;
    const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int32_t zz = ty; zz < 32; zz += kBlock / 32) {
        const int32_t z = z0 + zz, x = x0 + tx;
        if (z < nz && x < nx) tile[zz][tx] = in[((int64_t)z * ny + y) * nx + x];
    }
    __syncthreads();
    for (int32_t xx = ty; xx < 32; xx += kBlock / 32) {
        const int32_t x = x0 + xx, z = z0 + tx;
        if (z < nz && x < nx) out[((int64_t)y * nx + x) * nz + z] = tile[tx][xx];
    }
}

// out[z][y][x] += in[z][x][y]
__global__ __launch_bounds__(kBlock) void k_add_transposed_xy(const float* __restrict__ in, float* __restrict__ out,
                                                               int32_t nx, int32_t ny, int32_t ytiles)
{
    __shared__ float tile[32][33];
    const int32_t z = blockIdx.y / ytiles;
    const int32_t y0 = (blockIdx.y - z * ytiles) * 32, x0 = blockIdx.x * 32;
    const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t slab = (int64_t)z * nx * ny;
    for (int32_t xx = ty; xx < 32; xx += kBlock / 32) {
        const int32_t x = x0 + xx, y = y0 + tx;
        if (y < ny && x < nx) tile[xx][tx] = in[slab + (int64_t)x * ny + y];
    }
    __syncthreads();
    for (int32_t yy = ty; yy < 32; yy += kBlock / 32) {
        const int32_t y = y0 + yy, x = x0 + tx;
        if (y < ny && x < nx) out[slab + (int64_t)y * nx + x] += tile[tx][yy];
    }
}

// wt: per-ray weights applied to the sinogram values (the PET form), or none.
// imgT (one image, y fastest, zeroed) or NULL: views whose u axis runs along y add into
// it, to be added back transposed.
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_scatter(DevPlan P, const float* __restrict__ sino,
                                                     float* img, const float* __restrict__ wt, int64_t wt_stride,
                                                     float* imgT)
{
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.n_rays) return;
    const int64_t b = blockIdx.y;
    const double g = (double)sino[b * P.n_rays + r] * (wt != nullptr ? (double)wt[b * wt_stride + r] : 1.0);
    if (g == 0.0) return;
    Ray R;
    make_ray<DIM, MODE>(P, r, R);
    float* out = img + b * P.n_units;
    if (imgT != nullptr && view_prefers_y_fastest<MODE>(P, r)) {
        out = imgT;
        R.st[0] = P.ny;
        R.st[1] = 1;
    }
    ScatterVisit v{out, g * R.scale};
    walk<DIM>(P, R, v);
}

template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_counts(DevPlan P, int32_t first, int32_t n, double eps,
                                                    int32_t* __restrict__ counts)
{
    const int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (t >= n) return;
    Ray R;
    make_ray<DIM, MODE>(P, first + t, R);
    CountVisit v{eps / R.scale, 0};
    walk<DIM>(P, R, v);
    counts[t] = v.n;
}

// Entries [lo, hi) of a row in reverse order.
__device__ void reverse_entries(int32_t* __restrict__ idx, float* __restrict__ len, int32_t lo, int32_t hi)
{
    for (--hi; lo < hi; ++lo, --hi) {
        const int32_t a = idx[lo];
        idx[lo] = idx[hi];
        idx[hi] = a;
        const float b = len[lo];
        len[lo] = len[hi];
        len[hi] = b;
    }
}

// Sort a row written in order along the ray by 1D index I = (k ny + j) nx + i.  Along a
// line each of k, j and i is monotone, so the row is ordered lexicographically by
// (+-k, +-j, +-i) with the signs of the ray's direction: reversing the whole row where k
// falls, then every run of one k where j falls, then every run of one (k, j) where i
// falls sorts it.  A final insertion pass (no work on a sorted row) makes the order
// exact whatever the row's order was.
__device__ void sort_row(int32_t* __restrict__ idx, float* __restrict__ len, int32_t n, int32_t nx, int32_t nxy)
{
    const int32_t key[3] = {nxy, nx, 1};
    for (int lev = 0; lev < 3; ++lev) {
        const int32_t d = key[lev];
        for (int32_t a = 0; a < n;) {
            int32_t b = a + 1;
            if (lev > 0) {
                const int32_t run = idx[a] / key[lev - 1];
                while (b < n && idx[b] / key[lev - 1] == run) ++b;
            } else {
                b = n;
            }
            if (idx[a] / d > idx[b - 1] / d) reverse_entries(idx, len, a, b);
            a = b;
        }
    }
    for (int32_t m = 1; m < n; ++m) {
        const int32_t I = idx[m];
        const float l = len[m];
        int32_t q = m - 1;
        for (; q >= 0 && idx[q] > I; --q) {
            idx[q + 1] = idx[q];
            len[q + 1] = len[q];
        }
        idx[q + 1] = I;
        len[q + 1] = l;
    }
}

template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_hits(DevPlan P, int32_t first, int32_t n, double eps,
                                                  const int64_t* __restrict__ off,
                                                  int32_t* __restrict__ idx, float* __restrict__ len)
{
    const int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (t >= n) return;
    Ray R;
    make_ray<DIM, MODE>(P, first + t, R);
    const int64_t o = off[t];
    const int32_t cap = (int32_t)(off[t + 1] - o);
    EmitVisit v{idx + o, len + o, eps / R.scale, R.scale, 0, cap};
    walk<DIM>(P, R, v);
    // the order of the paper's hit lists (Algorithms 1 and 2; the tables of Sec. 5)
    sort_row(idx + o, len + o, v.n, P.nx, P.nx * P.ny);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(float* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = 0.0f;
}

// Dispatch a kernel template over (dim, mode).
template <template <int, int> class K, class... Args>
xrt_status dispatch(const DevPlan& P, dim3 grid, hipStream_t s, Args... args)
{
    auto go = [&](auto kern) -> xrt_status {
        hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, P, args...);
        return hip_fail(hipGetLastError(), "kernel launch");
    };
    if (P.dim == 2) {
        switch (P.mode) {
            case MODE_PARALLEL: return go(K<2, MODE_PARALLEL>::fn());
            case MODE_DIVERGENT: return go(K<2, MODE_DIVERGENT>::fn());
            case MODE_ARC: return go(K<2, MODE_ARC>::fn());
            default: return go(K<2, MODE_LIST>::fn());
        }
    }
    switch (P.mode) {
        case MODE_PARALLEL: return go(K<3, MODE_PARALLEL>::fn());
        case MODE_DIVERGENT: return go(K<3, MODE_DIVERGENT>::fn());
        case MODE_ARC: return go(K<3, MODE_ARC>::fn());
        default: return go(K<3, MODE_LIST>::fn());
    }
}

template <int D, int M> struct FwdK { static auto fn() { return k_forward<D, M, false>; } };
template <int D, int M> struct FwdNestK { static auto fn() { return k_forward<D, M, D == 3>; } };
template <int D, int M> struct FwdAttK { static auto fn() { return k_forward_att<D, M>; } };
template <int D, int M> struct FwdIlK { static auto fn() { return k_forward_il<D, M>; } };
template <int D, int M> struct FwdAttPairK { static auto fn() { return k_forward_att_pairs<D, M, false>; } };
template <int D, int M> struct FwdAttPairNestK { static auto fn() { return k_forward_att_pairs<D, M, D == 3>; } };
template <int D, int M> struct AdjAttK { static auto fn() { return k_adjoint_att<D, M>; } };
template <int D, int M> struct ScatK { static auto fn() { return k_scatter<D, M>; } };
template <int D, int M> struct CntK { static auto fn() { return k_counts<D, M>; } };
template <int D, int M> struct HitK { static auto fn() { return k_hits<D, M>; } };

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

xrt_status launch_fill_zero(float* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return XRT_OK;
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(kBlock), 0, s, dst, n);
    return hip_fail(hipGetLastError(), "fill kernel launch");
}

xrt_status launch_transpose_xy(const DevPlan& P, const float* img, float* imgT, hipStream_t s)
{
    const int32_t ytiles = (P.ny + 31) / 32;
    hipLaunchKernelGGL(k_transpose_xy, dim3((unsigned)((P.nx + 31) / 32), (unsigned)(ytiles * P.nz)), dim3(kBlock), 0,
                       s, img, imgT, P.nx, P.ny, ytiles);
    return hip_fail(hipGetLastError(), "transpose launch");
}

xrt_status launch_forward(const xrt_plan* p, const float* img, float* sino, int batch, hipStream_t s,
                          const float* wt, int64_t wt_stride)
{
    const DevPlan& P = p->dp;
    const uint64_t nb64 = (forward_threads(P) + kBlock - 1) / kBlock;
    if (nb64 > 0x7FFFFFF0ull) { set_error("forward launch too large"); return XRT_E_SIZE; }
    const uint32_t nb = (uint32_t)nb64;
    const uint32_t grid = P.xcd_remap ? (nb + 7u) / 8u * 8u : nb;
    // the walk's form (see walk()): chosen per plan
    // (column packets take the flat form: their lanes' z slopes differ, so the nested
    // form's inner loop would end at a different slab in every lane)
    auto launch = [&](dim3 g, const float* im, const float* imT, float* sn, const float* w, int64_t ws,
                      const float* imZ = nullptr) -> xrt_status {
        return P.nest_z && P.packet_cols != 1 ? dispatch<FwdNestK>(P, g, s, im, imT, sn, nb, w, ws, imZ)
                                              : dispatch<FwdK>(P, g, s, im, imT, sn, nb, w, ws, imZ);
    };
    if (P.dim == 3 && P.packet_cols == 1 && p->d_imgZ != nullptr) {
        for (int b = 0; b < batch; ++b) {
            const float* im = img + (int64_t)b * P.n_units;
            xrt_status st = launch_transpose_zfast(P, im, p->d_imgZ, s);
            if (st != XRT_OK) return st;
            st = launch(dim3(grid, 1u), im, (const float*)nullptr, sino + (int64_t)b * P.n_rays,
                        wt != nullptr ? wt + (int64_t)b * wt_stride : nullptr, (int64_t)0, p->d_imgZ);
            if (st != XRT_OK) return st;
        }
        return XRT_OK;
    }
    // one launch over the batch without the y-fastest copy (which holds one image) where
    // there is none, or for a batch of 2D images (small, so the copies would cost more
    // launches than they save); the values read are the same either way
    if (p->d_imgT == nullptr || (P.dim == 2 && batch > 1))
        return launch(dim3(grid, (unsigned)batch), img, (const float*)nullptr, sino, wt, wt_stride);
    for (int b = 0; b < batch; ++b) {
        const float* im = img + (int64_t)b * P.n_units;
        xrt_status st = launch_transpose_xy(P, im, p->d_imgT, s);
        if (st != XRT_OK) return st;
        st = launch(dim3(grid, 1u), im, (const float*)p->d_imgT, sino + (int64_t)b * P.n_rays,
                    wt != nullptr ? wt + (int64_t)b * wt_stride : nullptr, (int64_t)0);
        if (st != XRT_OK) return st;
    }
    return XRT_OK;
}

xrt_status launch_transpose_zfast(const DevPlan& P, const float* img, float* imgZ, hipStream_t s)
{
    const int32_t ztiles = (P.nz + 31) / 32;
    hipLaunchKernelGGL(k_transpose_zfast, dim3((unsigned)((P.nx + 31) / 32), (unsigned)(ztiles * P.ny)),
                       dim3(kBlock), 0, s, img, imgZ, P.nx, P.ny, P.nz, ztiles);
    return hip_fail(hipGetLastError(), "z-fastest transpose launch");
}

xrt_status launch_forward_batch(const DevPlan* hp, float* const* imgT, float* const* imgZ, const DevPlan* d_plans,
                                int32_t n, const int32_t* order, const float* const* imgs, float* const* sinos,
                                unsigned long long* counter, uint32_t grid, hipStream_t s)
{
    BatchQueue q{};
    BatchIO io{};
    q.n = n;
    int64_t chunk = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t m = order[k];
        const uint64_t nb = (forward_threads(hp[m]) + kBlock - 1) / kBlock;
        q.member[k] = m;
        q.first_chunk[k] = chunk;
        q.nblocks[k] = (int64_t)nb;
        chunk += ((int64_t)nb + kChunkBlocks - 1) / kChunkBlocks;
    }
    q.first_chunk[n] = chunk;
    for (int32_t m = 0; m < n; ++m) {
        io.in[m] = imgs[m];
        io.out[m] = sinos[m];
        io.inT[m] = imgT[m];
        io.inZ[m] = nullptr;
        if (hp[m].dim == 3 && hp[m].packet_cols == 1 && imgZ[m] != nullptr) {
            io.inT[m] = nullptr;
            io.inZ[m] = imgZ[m];
            xrt_status st = launch_transpose_zfast(hp[m], imgs[m], imgZ[m], s);
            if (st != XRT_OK) return st;
        } else if (imgT[m]) {
            xrt_status st = launch_transpose_xy(hp[m], imgs[m], imgT[m], s);
            if (st != XRT_OK) return st;
        }
    }
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
    xrt_status st = hip_fail(hipGetLastError(), "counter reset launch");
    if (st != XRT_OK) return st;
    const DevPlan& P0 = hp[0];
    if ((int64_t)grid > chunk) grid = (uint32_t)chunk;
    if (grid == 0) return XRT_OK;
    if (P0.dim == 3 && P0.mode == MODE_DIVERGENT)
        hipLaunchKernelGGL((k_forward_batch<3, MODE_DIVERGENT>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else if (P0.dim == 3 && P0.mode == MODE_PARALLEL)
        hipLaunchKernelGGL((k_forward_batch<3, MODE_PARALLEL>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else if (P0.dim == 3 && P0.mode == MODE_ARC)
        hipLaunchKernelGGL((k_forward_batch<3, MODE_ARC>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else if (P0.dim == 2 && P0.mode == MODE_DIVERGENT)
        hipLaunchKernelGGL((k_forward_batch<2, MODE_DIVERGENT>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else if (P0.dim == 2 && P0.mode == MODE_PARALLEL)
        hipLaunchKernelGGL((k_forward_batch<2, MODE_PARALLEL>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else if (P0.dim == 2 && P0.mode == MODE_ARC)
        hipLaunchKernelGGL((k_forward_batch<2, MODE_ARC>), dim3(grid), dim3(kBlock), 0, s, d_plans, q, io, counter);
    else {
        set_error("batched projection of ray lists is not supported");
        return XRT_E_UNSUPPORTED;
    }
    return hip_fail(hipGetLastError(), "batched forward launch");
}

uint32_t forward_batch_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_forward_batch<3, MODE_DIVERGENT>, kBlock, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 4;
    }
    return nb > 0 ? (uint32_t)nb : 1u;
}

xrt_status launch_forward_att(const xrt_plan* p, const float* img, const float* mu, int64_t mu_stride, float* sino,
                              int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    return dispatch<FwdAttK>(P, dim3(blocks_for(P.n_rays), (unsigned)batch), s, img, mu, mu_stride, sino);
}

xrt_status launch_forward_il(const xrt_plan* p, const float* img, float* sino, int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    return dispatch<FwdIlK>(P, dim3((unsigned)((P.n_rays + kBlock / 64 - 1) / (kBlock / 64))), s, img, sino,
                            (int32_t)batch);
}

xrt_status launch_forward_att_pairs(const xrt_plan* p, const float* img, const float* mu, int64_t mu_stride,
                                    float* sino, int batch, hipStream_t s)
{
    const DevPlan& P = p->dp;
    const unsigned pblocks = (unsigned)std::min<int64_t>((P.n_units + kBlock - 1) / kBlock, 65536);
    // column packets as in the plain forward (cone plans with 64 rows or more)
    const bool zp = P.dim == 3 && P.packet_cols == 1 && (P.mode == MODE_DIVERGENT || P.mode == MODE_ARC);
    for (int b = 0; b < batch; ++b) {
        if (zp) {
            const int32_t ztiles = (P.nz + 31) / 32;
            hipLaunchKernelGGL(k_att_pairs_zfast, dim3((unsigned)((P.nx + 31) / 32), (unsigned)(ztiles * P.ny)),
                               dim3(kBlock), 0, s, img + (int64_t)b * P.n_units, mu + (int64_t)b * mu_stride,
                               (float2*)p->d_att, P.nx, P.ny, P.nz, ztiles);
            xrt_status st = hip_fail(hipGetLastError(), "attenuation pairs launch");
            if (st != XRT_OK) return st;
            const uint64_t nb64 = (forward_threads(P) + kBlock - 1) / kBlock;
            if (nb64 > 0x7FFFFFF0ull) { set_error("attenuated forward launch too large"); return XRT_E_SIZE; }
            const dim3 g((unsigned)nb64);
            if (P.mode == MODE_DIVERGENT)
                hipLaunchKernelGGL((k_forward_att_pairs<3, MODE_DIVERGENT, false, true>), g, dim3(kBlock), 0, s, P,
                                   (const float*)p->d_att, sino + (int64_t)b * P.n_rays);
            else
                hipLaunchKernelGGL((k_forward_att_pairs<3, MODE_ARC, false, true>), g, dim3(kBlock), 0, s, P,
                                   (const float*)p->d_att, sino + (int64_t)b * P.n_rays);
            if ((st = hip_fail(hipGetLastError(), "kernel launch")) != XRT_OK) return st;
            continue;
        }
        hipLaunchKernelGGL(k_att_pairs, dim3(pblocks), dim3(kBlock), 0, s, img + (int64_t)b * P.n_units,
                           mu + (int64_t)b * mu_stride, (float2*)p->d_att, P.n_units);
        xrt_status st = hip_fail(hipGetLastError(), "attenuation pairs launch");
        if (st != XRT_OK) return st;
        st = P.nest_z ? dispatch<FwdAttPairNestK>(P, dim3(blocks_for(P.n_rays), 1u), s, (const float*)p->d_att,
                                                  sino + (int64_t)b * P.n_rays)
                      : dispatch<FwdAttPairK>(P, dim3(blocks_for(P.n_rays), 1u), s, (const float*)p->d_att,
                                              sino + (int64_t)b * P.n_rays);
        if (st != XRT_OK) return st;
    }
    return XRT_OK;
}

xrt_status launch_add_transposed_xy(const DevPlan& P, const float* imgT, float* img, hipStream_t s)
{
    const int32_t ytiles = (P.ny + 31) / 32;
    hipLaunchKernelGGL(k_add_transposed_xy, dim3((unsigned)((P.nx + 31) / 32), (unsigned)(ytiles * P.nz)),
                       dim3(kBlock), 0, s, imgT, img, P.nx, P.ny, ytiles);
    return hip_fail(hipGetLastError(), "transposed add launch");
}

// The scatters of 3D plans with a y-fastest workspace add the views whose u axis runs
// along y into it (zeroed first) and add it back transposed, one image at a time; the
// attenuated one also reads those views' map from a y-fastest copy (muT: n_units floats
// of plan workspace, or NULL to keep one layout).
xrt_status launch_adjoint_att(const xrt_plan* p, const float* sino, const float* mu, int64_t mu_stride, float* img,
                              int batch, hipStream_t s, float* muT)
{
    const DevPlan& P = p->dp;
    xrt_status st = launch_fill_zero(img, P.n_units * (int64_t)batch, s);
    if (st != XRT_OK) return st;
    if (P.dim != 3 || p->d_imgT == nullptr || muT == nullptr)
        return dispatch<AdjAttK>(P, dim3(blocks_for(P.n_rays), (unsigned)batch), s, sino, mu, mu_stride, img,
                                 (float*)nullptr, (const float*)nullptr);
    for (int b = 0; b < batch; ++b) {
        if ((st = launch_fill_zero(p->d_imgT, P.n_units, s)) != XRT_OK) return st;
        if ((st = launch_transpose_xy(P, mu + (int64_t)b * mu_stride, muT, s)) != XRT_OK) return st;
        st = dispatch<AdjAttK>(P, dim3(blocks_for(P.n_rays), 1u), s, sino + (int64_t)b * P.n_rays,
                               mu + (int64_t)b * mu_stride, (int64_t)0, img + (int64_t)b * P.n_units, p->d_imgT,
                               (const float*)muT);
        if (st != XRT_OK) return st;
        if ((st = launch_add_transposed_xy(P, p->d_imgT, img + (int64_t)b * P.n_units, s)) != XRT_OK) return st;
    }
    return XRT_OK;
}

xrt_status launch_adjoint_scatter(const xrt_plan* p, const float* sino, float* img, int batch,
                                  hipStream_t s, const float* wt, int64_t wt_stride)
{
    const DevPlan& P = p->dp;
    xrt_status st = launch_fill_zero(img, P.n_units * (int64_t)batch, s);
    if (st != XRT_OK) return st;
    if (P.dim != 3 || p->d_imgT == nullptr)
        return dispatch<ScatK>(P, dim3(blocks_for(P.n_rays), (unsigned)batch), s, sino, img, wt, wt_stride,
                               (float*)nullptr);
    for (int b = 0; b < batch; ++b) {
        if ((st = launch_fill_zero(p->d_imgT, P.n_units, s)) != XRT_OK) return st;
        st = dispatch<ScatK>(P, dim3(blocks_for(P.n_rays), 1u), s, sino + (int64_t)b * P.n_rays,
                             img + (int64_t)b * P.n_units, wt != nullptr ? wt + (int64_t)b * wt_stride : nullptr,
                             (int64_t)0, p->d_imgT);
        if (st != XRT_OK) return st;
        if ((st = launch_add_transposed_xy(P, p->d_imgT, img + (int64_t)b * P.n_units, s)) != XRT_OK) return st;
    }
    return XRT_OK;
}

xrt_status launch_hit_counts(const xrt_plan* p, int64_t first, int64_t n, double eps, int32_t* counts,
                             hipStream_t s)
{
    const DevPlan& P = p->dp;
    if (n <= 0) return XRT_OK;
    return dispatch<CntK>(P, dim3(blocks_for(n)), s, (int32_t)first, (int32_t)n, eps, counts);
}

xrt_status launch_hits(const xrt_plan* p, int64_t first, int64_t n, double eps, const int64_t* offsets,
                       int32_t* idx, float* len, hipStream_t s)
{
    const DevPlan& P = p->dp;
    if (n <= 0) return XRT_OK;
    return dispatch<HitK>(P, dim3(blocks_for(n)), s, (int32_t)first, (int32_t)n, eps, offsets, idx, len);
}

}  // namespace xrt
