// Rest-shape subspace on the device: the r lowest eigenvectors of H on the
// free vertices (section 5: U holds the eigenvectors of the rest global
// matrix with the smallest eigenvalues), by Chebyshev-filtered subspace
// iteration with Rayleigh-Ritz (the filter of Zhou and Saad, 2007):
//   repeat: Y <- p_d(H) Y with p_d the scaled Chebyshev polynomial that is 1
//           at 0 and small on [a, b] (a = largest Ritz value, b >= lambda_max);
//           orthonormalise Y (Cholesky QR, twice); Rayleigh-Ritz on Y^T H Y.
// Block products run in FP32 on the device (row-major N x m blocks); the
// m x m problems (Cholesky, symmetric eigenproblem) run in FP64 on the host.
// The result is an approximate eigenbasis (residual near the FP32 floor); the
// correction built from it stays an exact Galerkin projection because
// Lambda~ = U~^T H U~ is formed in FP64 from the stored values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "contact.hpp"
#include "scene.hpp"

namespace cloth {

namespace {

constexpr int GT = 32;  // Gram tile

// Y2 = alpha (H Y1 - c Y1) + beta Y0 on free rows (pinned rows 0); thread =
// (row, group of 4 columns); m % 4 == 0.  Y0 may be null (beta ignored).
__global__ void k_blk_cheb(int n, int m, const int* __restrict__ rp, const int* __restrict__ col,
                           const float* __restrict__ val, const uint8_t* __restrict__ pinned,
                           const float* __restrict__ Y1, const float* __restrict__ Y0, float* __restrict__ Y2,
                           float alpha, float c, float beta) {
    const int g4 = m >> 2;
    const size_t total = (size_t)n * g4;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int v = (int)(t / g4), q = (int)(t % g4);
        float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
        if (!pinned[v]) {
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int j = rp[v]; j < rp[v + 1]; ++j) {
                float a = val[j];
                float4 y = *reinterpret_cast<const float4*>(Y1 + (size_t)col[j] * m + 4 * q);
                acc.x += a * y.x;
                acc.y += a * y.y;
                acc.z += a * y.z;
                acc.w += a * y.w;
            }
            float4 y1 = *reinterpret_cast<const float4*>(Y1 + (size_t)v * m + 4 * q);
            out = make_float4(alpha * (acc.x - c * y1.x), alpha * (acc.y - c * y1.y), alpha * (acc.z - c * y1.z),
                              alpha * (acc.w - c * y1.w));
            if (Y0) {
                float4 y0 = *reinterpret_cast<const float4*>(Y0 + (size_t)v * m + 4 * q);
                out.x += beta * y0.x;
                out.y += beta * y0.y;
                out.z += beta * y0.z;
                out.w += beta * y0.w;
            }
        }
        *reinterpret_cast<float4*>(Y2 + (size_t)v * m + 4 * q) = out;
    }
}

// part[chunk][i][j] = sum over the chunk's rows of A[v][i] B[v][j] (FP64
// accumulation: the filtered blocks are ill-conditioned by design, and their
// Gram matrices must stay positive definite); block = (tile i, tile j,
// chunk), 32 x 32 outputs, 4 per thread.
__global__ void __launch_bounds__(256) k_blk_gram(int n, int m, const float* __restrict__ A,
                                                  const float* __restrict__ B, int nchunk, double* part) {
    __shared__ float as[GT][GT + 1];
    __shared__ float bs[GT][GT + 1];
    const int ti = blockIdx.x, tj = blockIdx.y, ch = blockIdx.z;
    const int per = (n + nchunk - 1) / nchunk;
    const int r0 = ch * per, r1 = min(n, r0 + per);
    const int tid = threadIdx.x;
    const int oy = (tid / 16) * 2, ox = (tid % 16) * 2;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int base = r0; base < r1; base += GT) {
        __syncthreads();
        for (int e = tid; e < GT * GT; e += 256) {
            int rr = e / GT, cc = e % GT;
            int v = base + rr;
            int ci = ti * GT + cc, cj = tj * GT + cc;
            as[rr][cc] = (v < r1 && ci < m) ? A[(size_t)v * m + ci] : 0.f;
            bs[rr][cc] = (v < r1 && cj < m) ? B[(size_t)v * m + cj] : 0.f;
        }
        __syncthreads();
        for (int rr = 0; rr < GT; ++rr) {
            double a0 = as[rr][oy], a1 = as[rr][oy + 1], b0 = bs[rr][ox], b1 = bs[rr][ox + 1];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            int i = ti * GT + oy + a, j = tj * GT + ox + b;
            if (i < m && j < m) part[(size_t)ch * m * m + (size_t)i * m + j] = acc[a][b];
        }
}

// Z = Y M with M (m x m, row-major FP32); thread = (row, 4 output columns)
__global__ void k_blk_rotate(int n, int m, const float* __restrict__ Y, const float* __restrict__ Mt,
                             float* __restrict__ Z) {
    const int g4 = m >> 2;
    const size_t total = (size_t)n * g4;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int v = (int)(t / g4), q = (int)(t % g4);
        const float* y = Y + (size_t)v * m;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int k = 0; k < m; ++k) {
            float a = y[k];
            float4 mm = *reinterpret_cast<const float4*>(Mt + (size_t)k * m + 4 * q);
            acc.x += a * mm.x;
            acc.y += a * mm.y;
            acc.z += a * mm.z;
            acc.w += a * mm.w;
        }
        *reinterpret_cast<float4*>(Z + (size_t)v * m + 4 * q) = acc;
    }
}

// initial block: hashed uniform values on free rows
__global__ void k_blk_init(int n, int m, const uint8_t* __restrict__ pinned, float* Y) {
    const size_t total = (size_t)n * m;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        uint64_t h = t * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        int v = (int)(t / m);
        Y[t] = pinned[v] ? 0.f : (float)((double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
}

// host: lower Cholesky of an SPD m x m matrix (in place), false if not SPD
bool chol(std::vector<double>& A, int m) {
    for (int k = 0; k < m; ++k) {
        double d = A[(size_t)k * m + k];
        for (int j = 0; j < k; ++j) d -= A[(size_t)k * m + j] * A[(size_t)k * m + j];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        A[(size_t)k * m + k] = d;
        for (int i = k + 1; i < m; ++i) {
            double s = A[(size_t)i * m + k];
            for (int j = 0; j < k; ++j) s -= A[(size_t)i * m + j] * A[(size_t)k * m + j];
            A[(size_t)i * m + k] = s / d;
        }
    }
    return true;
}

// host: symmetric eigen-decomposition by cyclic Jacobi rotations; A is
// destroyed, V (row-major, columns = eigenvectors) and w sorted ascending
void jacobi_eig(std::vector<double> A, int m, std::vector<double>& V, std::vector<double>& w) {
    V.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double a = A[(size_t)i * m + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {  // A <- J^T A J
                    double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - s * vkq;
                    V[(size_t)k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[(size_t)a * m + a] < A[(size_t)b * m + b]; });
    std::vector<double> Vs((size_t)m * m);
    w.resize(m);
    for (int c2 = 0; c2 < m; ++c2) {
        w[c2] = A[(size_t)idx[c2] * m + idx[c2]];
        for (int k = 0; k < m; ++k) Vs[(size_t)k * m + c2] = V[(size_t)k * m + idx[c2]];
    }
    V.swap(Vs);
}

#define HC(expr)                                                                                        \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) {                                                                         \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);                                    \
            return CLOTH_E_DEVICE;                                                                      \
        }                                                                                               \
    } while (0)

struct Work {
    float *Y = nullptr, *Y0 = nullptr, *Y1 = nullptr, *Z = nullptr, *M = nullptr;
    double* part = nullptr;
    bool owned = false;  // allocated here (freed on exit) or carved from a workspace
    ~Work() {
        if (!owned) return;
        for (float* p : {Y, Y0, Y1, Z, M})
            if (p) (void)hipFree(p);
        if (part) (void)hipFree(part);
    }
};

// Block width and Gram chunk count of the iteration for n rows and r wanted
// vectors.
int block_width(int r) { return ((r + std::max(8, r / 4)) + 3) / 4 * 4; }
int gram_chunks(int n) { return (int)std::max<int64_t>(1, std::min<int64_t>(64, n / 4096)); }
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace of the no-allocation entry point: a fixed array in device
// memory, one copy per GPU, held until the process ends.  In host code its
// name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[EIG_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Largest filter degree for which the scaled Chebyshev polynomial on [a, b]
// amplifies the lowest Ritz value theta_0 at most `growth` times more than
// the r-th one (|T_d(x)| grows as (x + sqrt(x^2 - 1))^d outside [-1, 1]):
// beyond that the wanted directions of the block collapse onto the lowest
// ones below the FP32 resolution of the block.
int filter_degree(double theta0, double thetar, double a, double b, int dmax, double growth) {
    const double e = 0.5 * (b - a), c = 0.5 * (b + a);
    auto g = [](double x) { return std::log(x + std::sqrt(std::max(0.0, x * x - 1.0))); };
    const double x0 = (c - theta0) / e, xr = (c - thetar) / e;
    if (!(x0 > 1.0) || !(xr >= 1.0) || !(g(x0) > g(xr))) return dmax;
    const double d = std::log(growth) / (g(x0) - g(xr));
    return (int)std::max(4.0, std::min((double)dmax, std::floor(d)));
}

}  // namespace

// Computes the basis into U (nv x r FP64, row-major, pinned rows zero) and
// the Ritz values into w.  Returns CLOTH_OK or an error with text in err.
size_t eig_workspace_bytes(int n, int r) {
    const int m = block_width(r), nchunk = gram_chunks(n);
    return 4 * align256(sizeof(float) * (size_t)n * m) + align256(sizeof(float) * (size_t)m * m) +
           align256(sizeof(double) * (size_t)nchunk * m * m);
}

cloth_status eig_static_workspace(void** out, std::string& err) {
    int dev = -1;
    HC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device ordinal out of range";
        return CLOTH_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        HC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            err = "hipGetSymbolAddress returned a null address for the basis workspace";
            return CLOTH_E_DEVICE;
        }
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return CLOTH_OK;
}

cloth_status device_eigenbasis(Scene& s, int r, int degree, int max_passes, double tol, std::vector<double>& U,
                               std::vector<double>& wout, int* passes_done, double* max_res, std::string& err,
                               void* workspace) {
    const int n = s.nv;
    const int m = block_width(r);
    const int nchunk = gram_chunks(n);
    Work w;
    size_t blk = sizeof(float) * (size_t)n * m;
    if (workspace) {
        // carve the buffers in eig_workspace_bytes' order; every one is
        // written before it is read, so nothing needs clearing
        unsigned char* p = static_cast<unsigned char*>(workspace);
        for (float** b : {&w.Y, &w.Y0, &w.Y1, &w.Z}) {
            *b = reinterpret_cast<float*>(p);
            p += align256(blk);
        }
        w.M = reinterpret_cast<float*>(p);
        p += align256(sizeof(float) * (size_t)m * m);
        w.part = reinterpret_cast<double*>(p);
    } else {
        w.owned = true;
        HC(hipMalloc(&w.Y, blk));
        HC(hipMalloc(&w.Y0, blk));
        HC(hipMalloc(&w.Y1, blk));
        HC(hipMalloc(&w.Z, blk));
        HC(hipMalloc(&w.M, sizeof(float) * (size_t)m * m));
        HC(hipMalloc(&w.part, sizeof(double) * (size_t)nchunk * m * m));
    }
    const int* rp = s.d.rowptr;
    const int* col = s.d.col;
    const float* val = s.d.val;
    const uint8_t* pin = s.d.pinned;
    const int grid = 4096, tpb = 256;
    // spectrum bound: Gershgorin on the host copy of H
    double bmax = 0.0;
    for (int v = 0; v < n; ++v) {
        double acc = 0.0;
        for (int j = s.rowptr[v]; j < s.rowptr[v + 1]; ++j) acc += std::fabs(s.val[j]);
        bmax = std::max(bmax, acc);
    }
    dim3 gg((m + GT - 1) / GT, (m + GT - 1) / GT, nchunk);
    std::vector<double> part((size_t)nchunk * m * m);
    auto gram = [&](const float* A, const float* B, std::vector<double>& G) -> cloth_status {
        hipLaunchKernelGGL(k_blk_gram, gg, dim3(256), 0, nullptr, n, m, A, B, nchunk, w.part);
        HC(hipGetLastError());
        HC(hipMemcpy(part.data(), w.part, sizeof(double) * part.size(), hipMemcpyDeviceToHost));
        G.assign((size_t)m * m, 0.0);
        for (int c = 0; c < nchunk; ++c)
            for (size_t e = 0; e < (size_t)m * m; ++e) G[e] += part[(size_t)c * m * m + e];
        return CLOTH_OK;
    };
    auto rotate = [&](const float* Y, const std::vector<double>& Mh, float* Z) -> cloth_status {
        std::vector<float> mf(Mh.begin(), Mh.end());
        HC(hipMemcpy(w.M, mf.data(), sizeof(float) * mf.size(), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_blk_rotate, dim3(grid), dim3(tpb), 0, nullptr, n, m, Y, w.M, Z);
        HC(hipGetLastError());
        return CLOTH_OK;
    };
    // orthonormalise Y in place (Cholesky QR twice): Y <- Y L^{-T}
    auto orth = [&]() -> cloth_status {
        for (int rep = 0; rep < 2; ++rep) {
            std::vector<double> G;
            cloth_status rc = gram(w.Y, w.Y, G);
            if (rc != CLOTH_OK) return rc;
            if (!chol(G, m)) {
                err = "Gram matrix of the block is not positive definite";
                return CLOTH_E_DIVERGED;
            }
            // Linv^T: solve L X = I, then transpose
            std::vector<double> Li((size_t)m * m, 0.0);
            for (int c = 0; c < m; ++c)
                for (int i = 0; i < m; ++i) {
                    double a = (i == c) ? 1.0 : 0.0;
                    for (int j = 0; j < i; ++j) a -= G[(size_t)i * m + j] * Li[(size_t)j * m + c];
                    Li[(size_t)i * m + c] = a / G[(size_t)i * m + i];
                }
            std::vector<double> Mh((size_t)m * m);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) Mh[(size_t)i * m + j] = Li[(size_t)j * m + i];
            rc = rotate(w.Y, Mh, w.Z);
            if (rc != CLOTH_OK) return rc;
            std::swap(w.Y, w.Z);
        }
        return CLOTH_OK;
    };
    std::vector<double> theta;
    // Rayleigh-Ritz: T = Y^T H Y, Y <- Y V; also leaves H Y (rotated) in Y1
    auto ritz = [&]() -> cloth_status {
        hipLaunchKernelGGL(k_blk_cheb, dim3(grid), dim3(tpb), 0, nullptr, n, m, rp, col, val, pin, w.Y,
                           (const float*)nullptr, w.Z, 1.0f, 0.0f, 0.0f);
        HC(hipGetLastError());
        std::vector<double> T;
        cloth_status rc = gram(w.Y, w.Z, T);
        if (rc != CLOTH_OK) return rc;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) {
                double a = 0.5 * (T[(size_t)i * m + j] + T[(size_t)j * m + i]);
                T[(size_t)i * m + j] = T[(size_t)j * m + i] = a;
            }
        std::vector<double> V;
        jacobi_eig(T, m, V, theta);
        rc = rotate(w.Y, V, w.Y1);
        if (rc != CLOTH_OK) return rc;
        std::swap(w.Y, w.Y1);
        rc = rotate(w.Z, V, w.Y1);  // H Y in the new basis
        return rc;
    };
    hipLaunchKernelGGL(k_blk_init, dim3(grid), dim3(tpb), 0, nullptr, n, m, pin, w.Y);
    HC(hipGetLastError());
    cloth_status rc = orth();
    if (rc != CLOTH_OK) return rc;
    rc = ritz();
    if (rc != CLOTH_OK) return rc;
    double res = 1e300;
    int p = 0;
    for (; p < max_passes; ++p) {
        // scaled Chebyshev filter on [a, b], normalised at 0
        const double a = theta[m - 1], b = bmax;
        const int deg = filter_degree(theta[0], theta[r - 1], a, b, degree, 1e4);
        const double e = 0.5 * (b - a), c = 0.5 * (b + a);
        double sig = e / (0.0 - c);
        const double tau = 2.0 / sig;
        // Y0 = Y, Y1 = (H Y - c Y) sig / e
        hipLaunchKernelGGL(k_blk_cheb, dim3(grid), dim3(tpb), 0, nullptr, n, m, rp, col, val, pin, w.Y,
                           (const float*)nullptr, w.Y1, (float)(sig / e), (float)c, 0.0f);
        HC(hipGetLastError());
        float* y0 = w.Y;
        float* y1 = w.Y1;
        float* y2 = w.Z;
        for (int i = 2; i <= deg; ++i) {
            double sn = 1.0 / (tau - sig);
            hipLaunchKernelGGL(k_blk_cheb, dim3(grid), dim3(tpb), 0, nullptr, n, m, rp, col, val, pin, y1, y0, y2,
                               (float)(2.0 * sn / e), (float)c, (float)(-sig * sn));
            float* t = y0;
            y0 = y1;
            y1 = y2;
            y2 = t;
            sig = sn;
        }
        HC(hipGetLastError());
        // the filtered block is in y1; make it Y (the other buffers are scratch)
        float* bufs[4] = {w.Y, w.Y0, w.Y1, w.Z};
        float* rest[3];
        int k2 = 0;
        for (float* q : bufs)
            if (q != y1) rest[k2++] = q;
        w.Y = y1;
        w.Y0 = rest[0];
        w.Y1 = rest[1];
        w.Z = rest[2];
        rc = orth();
        if (rc != CLOTH_OK) return rc;
        rc = ritz();
        if (rc != CLOTH_OK) return rc;
        // residual of the first r Ritz pairs: |H y - theta y| / theta (y unit)
        // ||H y - t y||^2 = (Hy.Hy) - 2 t (y.Hy) + t^2, from Grams in the Ritz basis
        std::vector<double> HH, YH;
        rc = gram(w.Y1, w.Y1, HH);
        if (rc != CLOTH_OK) return rc;
        res = 0.0;
        for (int i = 0; i < r; ++i) {
            double t = theta[i];
            double hh = HH[(size_t)i * m + i];
            double rr = std::sqrt(std::max(0.0, hh - t * t)) / std::max(t, 1e-300);
            res = std::max(res, rr);
        }
        if (res < tol) {
            ++p;
            break;
        }
    }
    std::vector<float> Yh((size_t)n * m);
    HC(hipMemcpy(Yh.data(), w.Y, blk, hipMemcpyDeviceToHost));
    U.assign((size_t)n * r, 0.0);
    for (int v = 0; v < n; ++v)
        if (!s.pinned[v])
            for (int c = 0; c < r; ++c) U[(size_t)v * r + c] = Yh[(size_t)v * m + c];
    wout.assign(theta.begin(), theta.begin() + r);
    if (passes_done) *passes_done = p;
    if (max_res) *max_res = res;
    return CLOTH_OK;
}

}  // namespace cloth
