// Inner projective-dynamics iteration kernels for gfx950 (wave64).
//
// One inner iteration (paper, Algorithm 1 inner loop; Eq. (local), (global),
// (subspace_collision), (high_frequency_residual)):
//   k_local_residual   local step (triangle strain projection; flat-rest
//                      bending adds no right-hand side) + inertia + collision
//                      targets; r0 = b - (H + diag W) x^k on free rows,
//                      evaluated in difference form; per-block partial
//                      products U^T r0 (r x 3)
//   k_reduce_g1        first level of the deterministic sum of the partials
//   k_solve_reduced    g = U^T r0 in FP64; without contact also q = Lambda~^{-1} g
//                      (with contact q = A^{-1} g follows on the contact factor)
//   k_expand           delta = U q  (x~ = x^k + delta)
//   k_jacobi_cheb      r1 = r0 - (H + diag W) delta, x^ = x~ + r1 / (diag H + W),
//                      Chebyshev blend -> x^{k+1}; max |x^{k+1} - x^k| in FP64
// Data: SoA FP32 positions (x, y, z planes of nv floats); the off-diagonal
// part of H in SELL-64 slices (one slice per wavefront, shared by the three
// coordinates) plus diag(H); U row-major in FP32 or BF16.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "friction.hpp"
#include "kernels.hpp"

namespace cloth {

namespace {

__device__ __forceinline__ float bf16_to_f32(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// Eight consecutive basis entries of row v starting at column c (c % 8 == 0).
template <typename UT>
__device__ __forceinline__ void load8(const UT* __restrict__ U, size_t off, float u[8]);

template <>
__device__ __forceinline__ void load8<float>(const float* __restrict__ U, size_t off, float u[8]) {
    const float4* p = reinterpret_cast<const float4*>(U + off);
    float4 a = p[0], b = p[1];
    u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
    u[4] = b.x; u[5] = b.y; u[6] = b.z; u[7] = b.w;
}

template <>
__device__ __forceinline__ void load8<uint16_t>(const uint16_t* __restrict__ U, size_t off, float u[8]) {
    uint4 a = *reinterpret_cast<const uint4*>(U + off);
    u[0] = __uint_as_float(a.x << 16); u[1] = __uint_as_float(a.x & 0xffff0000u);
    u[2] = __uint_as_float(a.y << 16); u[3] = __uint_as_float(a.y & 0xffff0000u);
    u[4] = __uint_as_float(a.z << 16); u[5] = __uint_as_float(a.z & 0xffff0000u);
    u[6] = __uint_as_float(a.w << 16); u[7] = __uint_as_float(a.w & 0xffff0000u);
}

// Eight consecutive basis entries kept in their stored form (16 bytes of
// BF16 or 32 bytes of FP32), so that many rows can be in flight at once.
template <typename UT>
struct RowChunk;

template <>
struct RowChunk<uint16_t> {
    uint4 a;
    __device__ __forceinline__ void load(const uint16_t* __restrict__ U, size_t off) {
        a = *reinterpret_cast<const uint4*>(U + off);
    }
    __device__ __forceinline__ void zero() { a = make_uint4(0u, 0u, 0u, 0u); }
    __device__ __forceinline__ void unpack(float u[8]) const {
        u[0] = __uint_as_float(a.x << 16); u[1] = __uint_as_float(a.x & 0xffff0000u);
        u[2] = __uint_as_float(a.y << 16); u[3] = __uint_as_float(a.y & 0xffff0000u);
        u[4] = __uint_as_float(a.z << 16); u[5] = __uint_as_float(a.z & 0xffff0000u);
        u[6] = __uint_as_float(a.w << 16); u[7] = __uint_as_float(a.w & 0xffff0000u);
    }
};

template <>
struct RowChunk<float> {
    float4 a, b;
    __device__ __forceinline__ void load(const float* __restrict__ U, size_t off) {
        const float4* p = reinterpret_cast<const float4*>(U + off);
        a = p[0];
        b = p[1];
    }
    __device__ __forceinline__ void zero() { a = b = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ __forceinline__ void unpack(float u[8]) const {
        u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
        u[4] = b.x; u[5] = b.y; u[6] = b.z; u[7] = b.w;
    }
};

// rows of U a lane keeps in flight (64 VGPRs of stored data)
template <typename UT>
constexpr int kRowsInFlight = sizeof(UT) == 2 ? 16 : 8;

// Closest 3x2 matrix with orthonormal columns: T = F (F^T F)^{-1/2}, with
// the 2x2 square root sqrt(S) = (S + sqrt(det S) I) / sqrt(tr S + 2 sqrt(det S)).
// F and T are row-major 3x2 (F[2*d + i]).
__device__ __forceinline__ void polar32(const float F[6], float T[6]) {
    float s00 = F[0] * F[0] + F[2] * F[2] + F[4] * F[4];
    float s01 = F[0] * F[1] + F[2] * F[3] + F[4] * F[5];
    float s11 = F[1] * F[1] + F[3] * F[3] + F[5] * F[5];
    float det = s00 * s11 - s01 * s01;
    if (!(det > 1e-20f)) {
        for (int i = 0; i < 6; ++i) T[i] = F[i];
        return;
    }
    float sd = sqrtf(det);
    float rden = 1.0f / sqrtf(s00 + s11 + 2.0f * sd);
    float r00 = (s00 + sd) * rden, r11 = (s11 + sd) * rden, r01 = s01 * rden;
    float isd = 1.0f / sd;
    float i00 = r11 * isd, i11 = r00 * isd, i01 = -r01 * isd;
    for (int d = 0; d < 3; ++d) {
        float f0 = F[2 * d], f1 = F[2 * d + 1];
        T[2 * d] = f0 * i00 + f1 * i01;
        T[2 * d + 1] = f0 * i01 + f1 * i11;
    }
}

// Strain-limited projection of a 3x2 deformation gradient: the nearest
// matrix whose singular values lie in [smin, smax], T = F M with
// M = V diag(c_i / sigma_i) V^T (F = U Sigma V^T, c_i = sigma_i clamped).
// M is the matrix function f(S) = clamp(sqrt(S)) / sqrt(S) of S = F^T F,
// formed from the two eigenvalues of S by spectral projectors:
// f(S) = f2 I + (f1 - f2) (S - l2 I) / (l1 - l2), which stays accurate when
// l1 - l2 is small (f1 - f2 is then small with it).
__device__ __forceinline__ void strain_limit32(const float F[6], float smin, float smax, float T[6]) {
    float s00 = F[0] * F[0] + F[2] * F[2] + F[4] * F[4];
    float s01 = F[0] * F[1] + F[2] * F[3] + F[4] * F[5];
    float s11 = F[1] * F[1] + F[3] * F[3] + F[5] * F[5];
    float det = s00 * s11 - s01 * s01;
    if (!(det > 1e-20f)) {
        for (int i = 0; i < 6; ++i) T[i] = F[i];
        return;
    }
    const float half_diff = 0.5f * (s00 - s11);
    const float disc = sqrtf(half_diff * half_diff + s01 * s01);   // (l1 - l2) / 2
    const float l1 = 0.5f * (s00 + s11) + disc;
    const float l2 = det / l1;
    const float g1 = sqrtf(l1), g2 = sqrtf(l2);
    const float f1 = fminf(fmaxf(g1, smin), smax) / g1;
    const float f2 = fminf(fmaxf(g2, smin), smax) / g2;
    const float b = disc > 0.f ? (f1 - f2) / (2.0f * disc) : 0.f;
    const float m00 = f2 + b * (s00 - l2), m11 = f2 + b * (s11 - l2), m01 = b * s01;
    for (int d = 0; d < 3; ++d) {
        float a0 = F[2 * d], a1 = F[2 * d + 1];
        T[2 * d] = a0 * m00 + a1 * m01;
        T[2 * d + 1] = a0 * m01 + a1 * m11;
    }
}

// Workgroups are dealt round-robin over the 8 XCDs; this maps workgroup b to
// a vertex tile so that each XCD (and its L2) works on one contiguous range,
// where the neighbour gathers of the SpMV and of the triangle stencils hit.
// It is a bijection of [0, nblk).
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    constexpr int X = 8;
    int x = b % X, i = b / X;
    int q = nblk / X, rem = nblk % X;
    return x * q + min(x, rem) + i;
}

// Off-diagonal row v of H in SELL-64: calls fn(H_vj, x4[j]) for its entries
// in storage order.  The column and value loads of C entries are issued
// together, then their C gathers, so that a row costs two dependent memory
// round trips per C entries instead of two per entry.  The slice width is
// common to the 64 rows of a wavefront, so the chunk bounds are uniform.
template <int C, typename Fn>
__device__ __forceinline__ void sell_row(const Dev& d, const float4* __restrict__ x4, int v, Fn&& fn) {
    const int lane = v & 63;
    const int p0 = d.sell_ptr[v >> 6], p1 = d.sell_ptr[(v >> 6) + 1];
    for (int j0 = p0 + lane; j0 < p1; j0 += 64 * C) {
        int col[C];
        float val[C];
#pragma unroll
        for (int b = 0; b < C; ++b) {
            const int j = j0 + 64 * b;
            col[b] = j < p1 ? d.sell_col[j] : v;
            val[b] = j < p1 ? d.sell_val[j] : 0.f;
        }
        float4 xc[C];
#pragma unroll
        for (int b = 0; b < C; ++b) xc[b] = x4[col[b]];
#pragma unroll
        for (int b = 0; b < C; ++b)
            if (j0 + 64 * b < p1) fn(val[b], xc[b]);
    }
}

// The same, for the short rows of cloth meshes (slices at most CA wide, the
// rest by sell_row): the wavefront's slice bounds come from scalar loads,
// the column and value loads of all CA entries are issued together, then
// their gathers in two batches (CB, then CA - CB), so that a row costs three
// dependent memory round trips.
template <int CA, int CB, typename Fn>
__device__ __forceinline__ void sell_row_short(const Dev& d, const float4* __restrict__ x4, int v, Fn&& fn) {
    const int lane = v & 63;
    const int slice = __builtin_amdgcn_readfirstlane(v >> 6);
    const int p0 = d.sell_ptr[slice], p1 = d.sell_ptr[slice + 1];
    int col[CA];
    float val[CA];
#pragma unroll
    for (int b = 0; b < CA; ++b) {
        const int jj = p0 + lane + 64 * b;
        col[b] = jj < p1 ? d.sell_col[jj] : v;
        val[b] = jj < p1 ? d.sell_val[jj] : 0.f;
    }
    {
        float4 xc[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) xc[b] = x4[col[b]];
#pragma unroll
        for (int b = 0; b < CB; ++b)
            if (p0 + lane + 64 * b < p1) fn(val[b], xc[b]);
    }
    {
        float4 xc[CA - CB];
#pragma unroll
        for (int b = CB; b < CA; ++b) xc[b - CB] = x4[col[b]];
#pragma unroll
        for (int b = CB; b < CA; ++b)
            if (p0 + lane + 64 * b < p1) fn(val[b], xc[b - CB]);
    }
    for (int j0 = p0 + lane + 64 * CA; j0 < p1; j0 += 64) fn(d.sell_val[j0], x4[d.sell_col[j0]]);
}

__device__ __forceinline__ double warp_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ bool gated(const int* g) { return g && *g; }

__device__ __forceinline__ double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }
// the value of a norm slot: the maximum over its sub-slots
__device__ __forceinline__ double slot_value(const unsigned long long* slot) {
    unsigned long long m = 0ull;
    for (int k = 0; k < DX_SUB; ++k) m = max(m, slot[8 * k]);
    return bits_to_double(m);
}

// block maximum of a per-thread value folded into *slot (FP64 bits; the
// values are non-negative, so their bit patterns order like the values)
__device__ __forceinline__ void block_max_to(double v, unsigned long long* slot) {
    __shared__ double wmax[TPB / 64];
    v = warp_max(v);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, wmax[i]);
        atomicMax(&slot[8 * (blockIdx.x % DX_SUB)], (unsigned long long)__double_as_longlong(m));
    }
}

}  // namespace

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Start of a step: the norm slots are cleared, the running step's status
// and iteration counters reset, the gates opened.
__global__ void k_step_open(unsigned long long* dxbits, int nslots, int* cnt, int* gate) {
    for (int i = threadIdx.x; i < nslots * DX_STRIDE; i += blockDim.x) dxbits[i] = 0ull;
    if (threadIdx.x == 0) {
        cnt[CNT_STEP_FAIL] = 0;
        cnt[CNT_INNER_DONE] = 0;
        cnt[CNT_OUTER_DONE] = 0;
        gate[0] = 0;
        gate[1] = 0;
    }
}

// Loop conditions of Algorithm 1 (tolerance mode), evaluated on the device
// before an inner iteration: the outer loop stops once the change of x over
// the previous outer block is below tol_out (prev_outer: that block's norm
// slot, -1 for the first block); the inner loop stops once the previous
// iteration's max |x^{k+1} - x^k| is below tol_in (prev_inner: its slot, -1
// for the first iteration of a block).  gate[1] = skip the block (set at its
// first iteration), gate[0] = skip this iteration.  block = 0 (residual
// forwarding): only the inner condition applies and nothing is counted.
__global__ void k_gate(int* gate, const unsigned long long* __restrict__ dxbits, int prev_inner, double tol_in,
                       int prev_outer, double tol_out, int block, int* cnt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (block && prev_inner < 0) {
        const int stop = prev_outer >= 0 && tol_out > 0 && slot_value(dxbits + (size_t)prev_outer * DX_STRIDE) < tol_out;
        gate[1] = stop;
        if (!stop) cnt[CNT_OUTER_DONE] += 1;
    }
    const int skip = (block && gate[1]) ||
                     (prev_inner >= 0 && tol_in > 0 && slot_value(dxbits + (size_t)prev_inner * DX_STRIDE) < tol_in);
    gate[0] = skip;
    if (block && !skip) cnt[CNT_INNER_DONE] += 1;
}

__global__ void k_copy3(float* __restrict__ dst, const float* __restrict__ src, int n3) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) dst[i] = src[i];
}

__global__ void k_aos4(const float* __restrict__ src, float4* __restrict__ dst, int n) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) dst[v] = make_float4(src[v], src[n + v], src[2 * n + v], 0.f);
}

// z = x* + h v* + h^2 g + 2 dx_rf (free rows), z = x* at pinned rows; x*
// saved.  Eq. (z) and, with a forwarded residual, Eq. (z_rf): the previous
// step's delta f = 2 M dx_rf / h^2 contributes h^2 M^{-1} delta f = 2 dx_rf.
__global__ void k_predict(Dev d, float h, float gx, float gy, float gz, const float* __restrict__ rfdx) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.nv) return;
    const int n = d.nv;
    bool pin = d.pinned[v] != 0;
    float g[3] = {gx, gy, gz};
    for (int c = 0; c < 3; ++c) {
        float xv = d.x[c * n + v];
        d.xstar[c * n + v] = xv;
        float zz = xv + h * d.v[c * n + v] + h * h * g[c];
        if (rfdx) zz += 2.0f * rfdx[c * n + v];
        d.z[c * n + v] = pin ? xv : zz;
    }
}

// Residual forwarding result: dx_rf = x_rf - x on free rows when the step's
// exiting t_TOI is below the threshold, else 0 (section 6).
__global__ void k_rf_finish(Dev d, const float* __restrict__ xrf, const float* __restrict__ x, float* rfdx,
                            const unsigned long long* __restrict__ t_last_bits, double rf_toi) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * d.nv) return;
    if (*d.fail) return;   // a failed step keeps the residual it started from
    double t = __longlong_as_double((long long)t_last_bits[0]);
    int v = i % d.nv;
    rfdx[i] = (t < rf_toi && !d.pinned[v]) ? xrf[i] - x[i] : 0.0f;
}

// x = x- + s (x+ - x-), x- <- x (the step-length filter, section 7).
// dxo (if set): max over vertices of |x - x-|, the change of x over the
// outer block (the outer loop condition of Algorithm 1), FP64.
__global__ void __launch_bounds__(TPB) k_filter(const int* __restrict__ gate, int nv, const float* __restrict__ xm,
                                                const float* __restrict__ xp, const double* __restrict__ s_dev,
                                                float* __restrict__ x, float* __restrict__ xm_out,
                                                unsigned long long* dxo) {
    if (gated(gate)) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    double s2 = 0.0;
    if (v < nv) {
        const float s = (float)s_dev[0];
        for (int c = 0; c < 3; ++c) {
            const int i = c * nv + v;
            const float a = xm[i];
            const float r = (s == 1.0f) ? xp[i] : a + s * (xp[i] - a);
            x[i] = r;
            xm_out[i] = r;
            const double dd = (double)r - (double)a;
            s2 += dd * dd;
        }
    }
    if (dxo) block_max_to(sqrt(s2), dxo);
}

// End of an outer block without contact: x = x^k, and the change of x over
// the block (max over vertices, FP64) into dxo.
__global__ void __launch_bounds__(TPB) k_block_end(const int* __restrict__ gate, int nv, const float* __restrict__ xk,
                                                   float* __restrict__ x, unsigned long long* dxo) {
    if (gated(gate)) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    double s2 = 0.0;
    if (v < nv) {
        for (int c = 0; c < 3; ++c) {
            const int i = c * nv + v;
            const float r = xk[i];
            const double dd = (double)r - (double)x[i];
            x[i] = r;
            s2 += dd * dd;
        }
    }
    block_max_to(sqrt(s2), dxo);
}

// v = (x - x*) / h.  A step whose status bits are set (a capacity overflow
// in a contact stage, a non-finite iterate, a tangle) is rolled back: x
// returns to x*, v keeps its value.  The step's status is published for the
// host (last step, and OR-ed into the record kept until the next stats read).
__global__ void k_epilogue(Dev d, float inv_h, int* cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = cnt[CNT_STEP_FAIL];
    if (i == 0) {
        cnt[CNT_LAST_STATUS] = f;
        atomicOr(&cnt[CNT_STICKY], f);
    }
    if (i >= 3 * d.nv) return;
    if (f)
        d.x[i] = d.xstar[i];
    else
        d.v[i] = (d.x[i] - d.xstar[i]) * inv_h;
}

// Local step, right-hand side b, residual r0 and the block's partial U^T r0.
// Thread = vertex; the elastic projection of each incident triangle is
// recomputed per corner so that accumulation is a deterministic gather.
// flags: bit 0 = contact terms (W, WY gathered here from the pair-constraint
// slots and the obstacle constraints, W stored for the later kernels),
// bit 1 = linear mode (b = 0: error propagation of the global iteration),
// bit 2 = every obstacle weight at k (a = 0; residual forwarding).
template <typename UT>
__global__ void __launch_bounds__(TPB) k_local_residual(Dev d, int flags) {
    __shared__ float sr[3][TPB];
    __shared__ float red[TPB * 24];
    if (gated(d.gate)) return;
    const int tid = threadIdx.x;
    const int n = d.nv;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int v = tile * TPB + tid;
    const bool contact = flags & 1, linear = flags & 2, force_k = flags & 4;
    const bool limited = !(d.smin == 1.0f && d.smax == 1.0f);
    // this thread's share of the block's U rows for U^T r0 (column group cg
    // of 8, vertices vg, vg + nvg, ...): the first PF rows are requested
    // now, so that they stream in while the local step runs
    const int r = d.r;
    const int ncg = r >> 3;
    const int nvg = TPB / ncg;
    const int cg = tid % ncg, vg = tid / ncg;
    const UT* U = static_cast<const UT*>(d.U);
    constexpr int PF = kRowsInFlight<UT>;
    RowChunk<UT> pre[PF];
#pragma unroll
    for (int b = 0; b < PF; ++b) {
        const int vv = vg + b * nvg;
        const int vtx = tile * TPB + vv;
        if (vg < nvg && vv < TPB && vtx < n) pre[b].load(U, (size_t)vtx * r + cg * 8);
        else pre[b].zero();
    }
    float r0[3] = {0.f, 0.f, 0.f};
    if (v < n) {
        const float* X = d.xk;
        const float4* X4 = d.x4;   // the same positions, AoS, for the gathers
        const float x0 = X[v], x1 = X[n + v], x2 = X[2 * n + v];
        // right-hand side minus the diagonal terms, accumulated as differences
        // (b - (M/h^2 + W) x) so that no large, nearly cancelling products
        // appear in FP32: inertia (m/h^2)(z - x), elastic projections, and the
        // collision corrections w (y - x)
        float bx = 0.f, by = 0.f, bz = 0.f;
        if (!linear) {
            float m = d.mh2[v];
            bx = m * (d.z[v] - x0);
            by = m * (d.z[n + v] - x1);
            bz = m * (d.z[2 * n + v] - x2);
            // incident triangles, CT at a time: their incidence codes, then
            // their records, then the corner positions are requested
            // together; the projections are summed in incidence order
            constexpr int CT = 2;
            for (int i = d.inc_ptr[v], e = d.inc_ptr[v + 1]; i < e; i += CT) {
                int code[CT];
#pragma unroll
                for (int b = 0; b < CT; ++b) code[b] = i + b < e ? d.inc[i + b] : 0;
                TriRec trs[CT];
#pragma unroll
                for (int b = 0; b < CT; ++b)
                    if (i + b < e) trs[b] = d.tri[code[b] >> 2];
                float4 qs[CT][3];
#pragma unroll
                for (int b = 0; b < CT; ++b)
                    if (i + b < e) {
                        qs[b][0] = X4[trs[b].v0];
                        qs[b][1] = X4[trs[b].v1];
                        qs[b][2] = X4[trs[b].v2];
                    }
#pragma unroll
                for (int b = 0; b < CT; ++b) {
                    if (i + b >= e) break;
                    const TriRec& tr = trs[b];
                    const int c = code[b] & 3;
                    const float4 q0 = qs[b][0], q1 = qs[b][1], q2 = qs[b][2];
                    float e1[3] = {q1.x - q0.x, q1.y - q0.y, q1.z - q0.z};
                    float e2[3] = {q2.x - q0.x, q2.y - q0.y, q2.z - q0.z};
                    float F[6], T[6];
                    for (int q = 0; q < 3; ++q) {
                        F[2 * q] = e1[q] * tr.gj0 + e2[q] * tr.gk0;
                        F[2 * q + 1] = e1[q] * tr.gj1 + e2[q] * tr.gk1;
                    }
                    if (limited)
                        strain_limit32(F, d.smin, d.smax, T);
                    else
                        polar32(F, T);
                    float g0, g1;
                    if (c == 0) {
                        g0 = -tr.gj0 - tr.gk0;
                        g1 = -tr.gj1 - tr.gk1;
                    } else if (c == 1) {
                        g0 = tr.gj0;
                        g1 = tr.gj1;
                    } else {
                        g0 = tr.gk0;
                        g1 = tr.gk1;
                    }
                    bx += tr.w * (T[0] * g0 + T[1] * g1);
                    by += tr.w * (T[2] * g0 + T[3] * g1);
                    bz += tr.w * (T[4] * g0 + T[5] * g1);
                }
            }
        }
        float Wv = 0.f;
        if (contact) {
            float wx = 0.f, wy = 0.f, wz = 0.f;
            for (int i = d.vslot_ptr[v], e = d.vslot_ptr[v + 1]; i < e; ++i) {
                float4 sl = d.slot[d.vslot[i]];   // (w, w (y - x))
                Wv += sl.x;
                wx += sl.y;
                wy += sl.z;
                wz += sl.w;
            }
            for (int j = 0; j < d.nob; ++j) {
                int a = d.ob_a[j * n + v];
                if (a < 0) continue;
                if (force_k) a = 0;
                float w = (d.Kb == 2.0f) ? ldexpf(d.kc, a) : d.kc * powf(d.Kb, (float)a);
                const ObstD& o = d.ob[j];
                double ox, oy, oz;
                const double rad = obstacle_radial(o, x0, x1, x2, ox, oy, oz);
                double sc = 0.0;   // y - x = (sc - 1) * radial
                if (rad - o.R < d.dhat && rad > 0) sc = (o.R + d.dhat) / rad - 1.0;
                Wv += w;
                wx += w * (float)(sc * ox);
                wy += w * (float)(sc * oy);
                wz += w * (float)(sc * oz);
                if (d.mu > 0.0f) {
                    double ux, uy, uz;
                    const double wf = obstacle_friction(d, o, w, ox, oy, oz, rad, x0, x1, x2, d.xstar[v],
                                                        d.xstar[n + v], d.xstar[2 * n + v], ux, uy, uz);
                    // weight wf toward the target x - u_T: w (y - x) = -wf u_T
                    Wv += (float)wf;
                    wx += (float)(-wf * ux);
                    wy += (float)(-wf * uy);
                    wz += (float)(-wf * uz);
                }
            }
            d.W[v] = Wv;
            if (!linear) {
                bx += wx;
                by += wy;
                bz += wz;
            }
        }
        if (!d.pinned[v]) {
            // off-diagonal part of H from the SELL-64 slices; elastic rows
            // sum to zero, so H x = (m/h^2) x + sum_{j != v} H_vj (x_j - x_v)
            float ax = 0.f, ay = 0.f, az = 0.f;
            if (!linear) {
                sell_row<5>(d, X4, v, [&](float a, float4 xc) {
                    ax += a * (xc.x - x0);
                    ay += a * (xc.y - x1);
                    az += a * (xc.z - x2);
                });
                r0[0] = bx - ax;
                r0[1] = by - ay;
                r0[2] = bz - az;
            } else {
                sell_row<5>(d, X4, v, [&](float a, float4 xc) {
                    ax += a * xc.x;
                    ay += a * xc.y;
                    az += a * xc.z;
                });
                const float dv = d.diag[v] + Wv;
                r0[0] = -ax - dv * x0;
                r0[1] = -ay - dv * x1;
                r0[2] = -az - dv * x2;
            }
        }
        // d.b holds r0 = b - (H + diag W) x^k for the Jacobi sweep
        d.b[v] = r0[0];
        d.b[n + v] = r0[1];
        d.b[2 * n + v] = r0[2];
    }
    sr[0][tid] = r0[0];
    sr[1][tid] = r0[1];
    sr[2][tid] = r0[2];
    __syncthreads();
    // partial U^T r0 over this block's vertices: thread = (column group of 8, vertex group)
    float acc[8][3];
    for (int i = 0; i < 8; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.f;
    if (vg < nvg) {
#pragma unroll
        for (int b = 0; b < PF; ++b) {
            const int vv = vg + b * nvg;
            if (vv >= TPB) break;
            float u[8];
            pre[b].unpack(u);
            float a0 = sr[0][vv], a1 = sr[1][vv], a2 = sr[2][vv];
            for (int i = 0; i < 8; ++i) {
                acc[i][0] += u[i] * a0;
                acc[i][1] += u[i] * a1;
                acc[i][2] += u[i] * a2;
            }
        }
        // the remaining rows (r > 128 BF16 / 64 FP32) in batches of 4
        for (int vv0 = vg + PF * nvg; vv0 < TPB; vv0 += 4 * nvg) {
            float u[4][8];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int vv = vv0 + b * nvg;
                const int vtx = tile * TPB + vv;
                if (vv < TPB && vtx < n) {
                    load8<UT>(U, (size_t)vtx * r + cg * 8, u[b]);
                } else {
                    for (int i = 0; i < 8; ++i) u[b][i] = 0.f;
                }
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int vv = vv0 + b * nvg;
                if (vv >= TPB) break;
                float a0 = sr[0][vv], a1 = sr[1][vv], a2 = sr[2][vv];
                for (int i = 0; i < 8; ++i) {
                    acc[i][0] += u[b][i] * a0;
                    acc[i][1] += u[b][i] * a1;
                    acc[i][2] += u[b][i] * a2;
                }
            }
        }
        for (int i = 0; i < 8; ++i)
            for (int c = 0; c < 3; ++c) red[vg * (r * 3) + (cg * 8 + i) * 3 + c] = acc[i][c];
    }
    __syncthreads();
    for (int o = tid; o < r * 3; o += TPB) {
        float s = 0.f;
        for (int g = 0; g < nvg; ++g) s += red[g * (r * 3) + o];
        d.gpart[(size_t)tile * (r * 3) + o] = s;
    }
}

// First reduction level: block s sums partial rows [s*SEG, (s+1)*SEG) in FP64.
constexpr int SEG = U_SEG;
__global__ void k_reduce_g1(const int* __restrict__ gate, const float* __restrict__ gpart, int nblk, int m,
                            double* __restrict__ out) {
    if (gated(gate)) return;
    int s = blockIdx.x;
    int b0 = s * SEG, b1 = min(nblk, b0 + SEG);
    for (int o = threadIdx.x; o < m; o += blockDim.x) {
        double acc = 0.0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) acc += (double)gpart[(size_t)b * m + o];
        out[(size_t)s * m + o] = acc;
    }
}

// g = sum of the level-1 partials (FP64) -> d.gvec; without contact also
// q = A^{-1} g with the precomputed inverse of Lambda~: one wavefront per
// row of A^{-1} at a time, lanes over its columns (coalesced), three
// right-hand sides reduced across the wavefront.
__global__ void __launch_bounds__(1024) k_solve_reduced(Dev d, const double* __restrict__ g1, int nseg, int solve) {
    extern __shared__ double gs[];
    if (gated(d.gate)) return;
    const int r = d.r, m = r * 3;
    for (int o = threadIdx.x; o < m; o += blockDim.x) {
        double acc = 0.0;
#pragma unroll 8
        for (int s = 0; s < nseg; ++s) acc += g1[(size_t)s * m + o];
        gs[o] = acc;
        d.gvec[o] = acc;
    }
    __syncthreads();
    if (!solve) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wave; c < r; c += nw) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int j = lane; j < r; j += 64) {
            double a = d.Ainv[(size_t)c * r + j];
            a0 += a * gs[j * 3];
            a1 += a * gs[j * 3 + 1];
            a2 += a * gs[j * 3 + 2];
        }
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o);
            a1 += __shfl_xor(a1, o);
            a2 += __shfl_xor(a2, o);
        }
        if (lane == 0) {
            d.Qd[c * 3] = a0;
            d.Qd[c * 3 + 1] = a1;
            d.Qd[c * 3 + 2] = a2;
            d.Qf[c * 3] = (float)a0;
            d.Qf[c * 3 + 1] = (float)a1;
            d.Qf[c * 3 + 2] = (float)a2;
        }
    }
}

// delta = U q into d.d4 (AoS, gathered by the Jacobi sweep); add = 1:
// d.xt = x^k + U q (SoA).
// G lanes share one row of U (G = r/8 rounded up to a power of two), each
// lane holding the q entries of its 8 columns in registers, so that a
// wavefront reads 64/G whole rows per load: contiguous runs of U instead of
// one 16-byte piece of 64 different rows.  The per-row sums are reduced
// across the G lanes and staged in LDS for a coalesced store.
template <typename UT>
__global__ void __launch_bounds__(TPB) k_expand(Dev d, int add) {
    __shared__ float res[3][TPB];
    if (gated(d.gate)) return;
    const int r = d.r, ncg = r >> 3;
    int G = 1;
    while (G < ncg) G <<= 1;               // r <= 256: G <= 32
    const int per = 64 / G;                // rows per wavefront per round
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cg = lane % G, vs = lane / G;
    const bool active = cg < ncg;
    float q[8][3];
    for (int i = 0; i < 8; ++i)
        for (int k = 0; k < 3; ++k) q[i][k] = active ? d.Qf[(cg * 8 + i) * 3 + k] : 0.f;
    const int n = d.nv;
    const int base = xcd_tile(blockIdx.x, gridDim.x) * TPB + wave * 64;
    const UT* U = static_cast<const UT*>(d.U);
    // rounds in batches of PF: all loads of a batch (one row per round, PF
    // rounds: 16 rows of BF16 or 8 of FP32 per lane) are issued before their
    // products, so that each lane keeps that many rows in flight
    constexpr int PF = kRowsInFlight<UT>;
    for (int rnd0 = 0; rnd0 < G; rnd0 += PF) {
        RowChunk<UT> raw[PF];
#pragma unroll
        for (int b = 0; b < PF; ++b) {
            const int v = base + (rnd0 + b) * per + vs;
            if (rnd0 + b < G && active && v < n) raw[b].load(U, (size_t)v * r + cg * 8);
            else raw[b].zero();
        }
#pragma unroll
        for (int b = 0; b < PF; ++b) {
            if (rnd0 + b >= G) break;
            const int lv = (rnd0 + b) * per + vs;
            float u[8];
            raw[b].unpack(u);
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
            for (int i = 0; i < 8; ++i) {
                a0 += u[i] * q[i][0];
                a1 += u[i] * q[i][1];
                a2 += u[i] * q[i][2];
            }
            for (int o = 1; o < G; o <<= 1) {
                a0 += __shfl_xor(a0, o);
                a1 += __shfl_xor(a1, o);
                a2 += __shfl_xor(a2, o);
            }
            if (cg == 0) {
                res[0][wave * 64 + lv] = a0;
                res[1][wave * 64 + lv] = a1;
                res[2][wave * 64 + lv] = a2;
            }
        }
    }
    __syncthreads();
    const int v = base - wave * 64 + tid;
    if (v >= n) return;
    if (add) {
        d.xt[v] = d.xk[v] + res[0][tid];
        d.xt[n + v] = d.xk[n + v] + res[1][tid];
        d.xt[2 * n + v] = d.xk[2 * n + v] + res[2][tid];
    } else {
        d.d4[v] = make_float4(res[0][tid], res[1][tid], res[2][tid], 0.f);
    }
}

// delta = U q on the matrix cores for a BF16 basis (v_mfma_f32_16x16x32_bf16:
// 16 vertices x 32 basis columns of U against 32 x 16 of q, whose columns
// 0..2 are the coordinates and the rest zero).  q (FP32) is split into three
// BF16 parts hi + mid + lo that sum to it exactly, so the three products add
// up to U~ q with FP32 accumulation.  The contraction order over the basis
// columns is free, so lane group g = l / 16 (of the A operand) takes the NC
// chunks of 8 columns [8 NC g, 8 NC (g + 1)) of its row: a lane reads 16 NC
// contiguous bytes of one row, four lanes cover the row (r <= 32 NC).
// A wavefront takes 16-vertex tiles of its workgroup's 256 vertices.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int NC>
__global__ void __launch_bounds__(TPB) k_expand_mfma(Dev d, int add) {
    __shared__ uint4 frag[3][NC][64];   // B operands, in lane order
    __shared__ float res[TPB / 64][3][64];
    if (gated(d.gate)) return;
    const int r = d.r;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int n = d.nv;
    // B operands: q's three BF16 parts for lane l's column l % 16 and rows
    // k = 8 NC (l / 16) + 8 c + i, staged once per workgroup
    for (int e = tid; e < NC * 64; e += TPB) {
        const int c = e / 64, l = e % 64, gl = l >> 4, jl = l & 15;
        uint32_t w[3][4];
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            uint32_t h2[3] = {0u, 0u, 0u};
#pragma unroll
            for (int i2 = 0; i2 < 2; ++i2) {
                const int k = 8 * NC * gl + 8 * c + i + i2;
                const float q = (jl < 3 && k < r) ? d.Qf[k * 3 + jl] : 0.f;
                const uint32_t h = f32_to_bf16_rne(q);
                const float qh = __uint_as_float(h << 16);
                const uint32_t m = f32_to_bf16_rne(q - qh);
                const float qm = __uint_as_float(m << 16);
                const uint32_t lo = f32_to_bf16_rne(q - qh - qm);
                h2[0] |= h << (16 * i2);
                h2[1] |= m << (16 * i2);
                h2[2] |= lo << (16 * i2);
            }
#pragma unroll
            for (int p = 0; p < 3; ++p) w[p][i / 2] = h2[p];
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) frag[p][c][l] = make_uint4(w[p][0], w[p][1], w[p][2], w[p][3]);
    }
    const int base = xcd_tile(blockIdx.x, gridDim.x) * TPB + wave * 64;
    const uint16_t* U = static_cast<const uint16_t*>(d.U);
    const int col0 = 8 * NC * g;
    // the A operands of the wavefront's four tiles, two tiles in flight:
    // tile t + 2 is requested before tile t is multiplied
    uint4 a[2][NC];
    auto load_tile = [&](int t, uint4 (&buf)[NC]) {
        const int v = base + 16 * t + j;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int k = col0 + 8 * c;
            if (v < n && k < r) buf[c] = *reinterpret_cast<const uint4*>(U + (size_t)v * r + k);
            else buf[c] = make_uint4(0u, 0u, 0u, 0u);
        }
    };
    load_tile(0, a[0]);
    load_tile(1, a[1]);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bf16x8_t av = __builtin_bit_cast(bf16x8_t, a[t & 1][c]);
#pragma unroll
            for (int p = 0; p < 3; ++p)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8_t, frag[p][c][lane]),
                                                              acc, 0, 0, 0);
        }
        if (t + 2 < 4) load_tile(t + 2, a[t & 1]);
        // lane (g, j < 3) holds coordinate j of the tile's vertices 4 g + e
        if (j < 3)
#pragma unroll
            for (int e = 0; e < 4; ++e) res[wave][j][16 * t + 4 * g + e] = acc[e];
    }
    __syncthreads();
    const int v = base + lane;
    if (v >= n) return;
    if (add) {
        d.xt[v] = d.xk[v] + res[wave][0][lane];
        d.xt[n + v] = d.xk[n + v] + res[wave][1][lane];
        d.xt[2 * n + v] = d.xk[2 * n + v] + res[wave][2][lane];
    } else {
        d.d4[v] = make_float4(res[wave][0][lane], res[wave][1][lane], res[wave][2][lane], 0.f);
    }
}

// Jacobi sweep on the residual of x~ = x^k + delta with the Chebyshev blend:
//   r1 = r0 - (H + diag W) delta   (= b - (H + diag W) x~, by linearity),
//   x^ - x^k = delta + r1 / (diag H + W) = (r0 - offdiag(H) delta) / (diag H + W),
//   x^{k+1} = x^{k-1} + omega (gamma (x^ - x^k) + x^k - x^{k-1}).
// d.b holds r0 and d.d4 holds delta = U q; x^{k+1} is written SoA to d.xk1
// and AoS to d.x4 (the next local step's gathers).  A non-finite change
// flags the step as diverged.  Gated (a converged loop): x^{k+1} = x^k and
// the slot repeats the previous iteration's norm (dx_prev).
// Rank-2 A-Jacobi (sec. 8.1), two damped Jacobi steps per iteration, as two
// launches: mode 1 writes e1 = gamma (x^ - x^k) to d.e4 (y1 = x^k + e1);
// mode 2 repeats the sweep with e1 in place of delta, whose x^ - x^k is then
// e1 + D^{-1} (b - A y1), and writes x^{k+1} = y1 + gamma D^{-1} (b - A y1).
__global__ void __launch_bounds__(TPB) k_jacobi_cheb(Dev d, float omega, float gamma, int has_contact,
                                                    unsigned long long* dx_slot,
                                                    const unsigned long long* __restrict__ dx_prev, int mode) {
    const int n = d.nv;
    const int v = xcd_tile(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    if (gated(d.gate)) {
        if (mode == 1) return;
        if (v < n)
            for (int c = 0; c < 3; ++c) d.xk1[c * n + v] = d.xk[c * n + v];
        if (blockIdx.x == 0 && threadIdx.x < DX_SUB && dx_prev) dx_slot[8 * threadIdx.x] = dx_prev[8 * threadIdx.x];
        return;
    }
    double dxm = 0.0;
    if (v < n) {
        const float4* DL = mode == 2 ? d.e4 : d.d4;
        float xk[3] = {d.xk[v], d.xk[n + v], d.xk[2 * n + v]};
        float xkm1[3] = {d.xkm1[v], d.xkm1[n + v], d.xkm1[2 * n + v]};
        float dh[3] = {0.f, 0.f, 0.f};
        if (!d.pinned[v]) {
            // the row's own data is requested before the gathers
            const float r00 = d.b[v], r01 = d.b[n + v], r02 = d.b[2 * n + v];
            const float dg = d.diag[v] + (has_contact ? d.W[v] : 0.f);
            float ax = 0.f, ay = 0.f, az = 0.f;
            sell_row_short<12, 8>(d, DL, v, [&](float a, float4 dc) {
                ax += a * dc.x;
                ay += a * dc.y;
                az += a * dc.z;
            });
            float inv = 1.0f / dg;
            // x^ - x^k = delta + (r0 - (H + diag W) delta) / (diag H + W)
            //          = (r0 - offdiag(H) delta) / (diag H + W)
            dh[0] = (r00 - ax) * inv;
            dh[1] = (r01 - ay) * inv;
            dh[2] = (r02 - az) * inv;
        }
        if (mode == 1) {
            d.e4[v] = make_float4(gamma * dh[0], gamma * dh[1], gamma * dh[2], 0.f);
            return;
        }
        double s2 = 0.0;
        float nx[3];
        const float4 e1 = mode == 2 ? d.e4[v] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float e1c[3] = {e1.x, e1.y, e1.z};
        for (int c = 0; c < 3; ++c) {
            if (mode == 2)
                nx[c] = (xk[c] + e1c[c]) + gamma * (dh[c] - e1c[c]);
            else
                nx[c] = xkm1[c] + omega * (gamma * dh[c] + (xk[c] - xkm1[c]));
            d.xk1[c * n + v] = nx[c];
            double dd = (double)nx[c] - (double)xk[c];
            s2 += dd * dd;
        }
        d.x4[v] = make_float4(nx[0], nx[1], nx[2], 0.f);   // gather copy for the next local step
        dxm = sqrt(s2);
        if (!(dxm <= 1.0e300) && d.fail) atomicOr(d.fail, STEP_DIVERGED);
    }
    block_max_to(dxm, dx_slot);
}

// ------------------------------------------------------------ launchers

static inline int blocks_for(int n) { return (n + TPB - 1) / TPB; }

namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

template <typename... KArgs, typename... Args>
void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args) {
    if (t_ev_start && t_ev_stop)
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, t_ev_start, t_ev_stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
}
}  // namespace

void set_kernel_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

void clear_kernel_events() {
    t_ev_start = nullptr;
    t_ev_stop = nullptr;
}

bool kernel_events(hipEvent_t* start, hipEvent_t* stop) {
    *start = t_ev_start;
    *stop = t_ev_stop;
    return t_ev_start && t_ev_stop;
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_copy3(float* dst, const float* src, int nv, hipStream_t st) {
    hipLaunchKernelGGL(k_copy3, dim3(blocks_for(3 * nv)), dim3(TPB), 0, st, dst, src, 3 * nv);
    return hipGetLastError();
}

hipError_t launch_aos4(const float* src, float4* dst, int nv, hipStream_t st) {
    hipLaunchKernelGGL(k_aos4, dim3(blocks_for(nv)), dim3(TPB), 0, st, src, dst, nv);
    return hipGetLastError();
}

hipError_t launch_predict(const Dev& d, float h, float gx, float gy, float gz, const float* rfdx, hipStream_t st) {
    hipLaunchKernelGGL(k_predict, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, h, gx, gy, gz, rfdx);
    return hipGetLastError();
}

hipError_t launch_rf_finish(const Dev& d, const float* xrf, const float* x, float* rfdx,
                            const unsigned long long* t_last_bits, double rf_toi, hipStream_t st) {
    hipLaunchKernelGGL(k_rf_finish, dim3(blocks_for(3 * d.nv)), dim3(TPB), 0, st, d, xrf, x, rfdx, t_last_bits,
                       rf_toi);
    return hipGetLastError();
}

hipError_t launch_filter(const Dev& d, const float* xm, const float* xp, const double* s_dev, float* x,
                         float* xm_out, unsigned long long* dxo, hipStream_t st) {
    hipLaunchKernelGGL(k_filter, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d.gate, d.nv, xm, xp, s_dev, x,
                       xm_out, dxo);
    return hipGetLastError();
}

hipError_t launch_block_end(const Dev& d, unsigned long long* dxo, hipStream_t st) {
    hipLaunchKernelGGL(k_block_end, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d.gate, d.nv, (const float*)d.xk, d.x,
                       dxo);
    return hipGetLastError();
}

hipError_t launch_epilogue(const Dev& d, float inv_h, int* cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_epilogue, dim3(blocks_for(3 * d.nv)), dim3(TPB), 0, st, d, inv_h, cnt);
    return hipGetLastError();
}

hipError_t launch_step_open(unsigned long long* dxbits, int nslots, int* cnt, int* gate, hipStream_t st) {
    hipLaunchKernelGGL(k_step_open, dim3(1), dim3(256), 0, st, dxbits, nslots, cnt, gate);
    return hipGetLastError();
}

hipError_t launch_gate(int* gate, const unsigned long long* dxbits, int prev_inner, double tol_in, int prev_outer,
                       double tol_out, int block, int* cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_gate, dim3(1), dim3(64), 0, st, gate, dxbits, prev_inner, tol_in, prev_outer, tol_out, block,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_local_residual(const Dev& d, int prec, int flags, hipStream_t st) {
    if (prec == CLOTH_MIXED)
        launch_timed(k_local_residual<uint16_t>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, flags);
    else
        launch_timed(k_local_residual<float>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, flags);
    return hipGetLastError();
}

hipError_t launch_reduce_solve(const Dev& d, int nblk, int contact, double* gpart2, hipStream_t st) {
    const int m = d.r * 3;
    int nseg = (nblk + SEG - 1) / SEG;
    hipLaunchKernelGGL(k_reduce_g1, dim3(nseg), dim3(256), 0, st, d.gate, (const float*)d.gpart, nblk, m, gpart2);
    // the second level (g in d.gvec), and without contact the solve with the
    // inverse of Lambda~; with contact the solve on the contact factor
    // follows once it is ready, and g is summed here, before that wait
    hipLaunchKernelGGL(k_solve_reduced, dim3(1), dim3(1024), sizeof(double) * m, st, d,
                       (const double*)gpart2, nseg, contact ? 0 : 1);
    return hipGetLastError();
}

hipError_t launch_expand(const Dev& d, int prec, int add, hipStream_t st) {
    const int nc = (d.r + 31) / 32;   // 8-column chunks per lane (r <= 32 nc)
    if (prec == CLOTH_MIXED && nc <= 1)
        launch_timed(k_expand_mfma<1>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, add);
    else if (prec == CLOTH_MIXED && nc <= 2)
        launch_timed(k_expand_mfma<2>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, add);
    else if (prec == CLOTH_MIXED && nc <= 4)
        launch_timed(k_expand_mfma<4>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, add);
    else if (prec == CLOTH_MIXED)
        launch_timed(k_expand_mfma<6>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, add);
    else
        launch_timed(k_expand<float>, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, add);
    return hipGetLastError();
}

hipError_t launch_jacobi_cheb(const Dev& d, float omega, float gamma, int has_contact,
                              unsigned long long* dx_slot, const unsigned long long* dx_prev, hipStream_t st,
                              int mode) {
    launch_timed(k_jacobi_cheb, dim3(blocks_for(d.nv)), dim3(TPB), 0, st, d, omega, gamma, has_contact, dx_slot,
                 dx_prev, mode);
    return hipGetLastError();
}

}  // namespace cloth
