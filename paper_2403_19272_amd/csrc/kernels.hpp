// Launch wrappers of the cloth kernels (device code in pd_kernels.hip and
// contact_kernels.hip).  All enqueue on `st` and return the launch status.
#pragma once

#include "scene.hpp"

namespace cloth {

// Kernel-level timing: while a pair is set (on this host thread), the
// single-kernel launchers below (local residual, expand, Jacobi sweep)
// launch through hipExtLaunchKernelGGL with these events, which then carry
// the kernel's own start and end time instead of a marker around it.
void set_kernel_events(hipEvent_t start, hipEvent_t stop);
void clear_kernel_events();
// the pair set on this thread, if any (for launchers in other files)
bool kernel_events(hipEvent_t* start, hipEvent_t* stop);

// ---- PD iteration (pd_kernels.hip)
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t st);
hipError_t launch_copy3(float* dst, const float* src, int nv, hipStream_t st);
// AoS float4 copy of an SoA position vector (gather copy of x^k)
hipError_t launch_aos4(const float* src, float4* dst, int nv, hipStream_t st);
hipError_t launch_predict(const Dev& d, float h, float gx, float gy, float gz, const float* rfdx, hipStream_t st);
hipError_t launch_rf_finish(const Dev& d, const float* xrf, const float* x, float* rfdx,
                            const unsigned long long* t_last_bits, double rf_toi, hipStream_t st);
// x = xm + s (xp - xm) into x and xm_out; dxo (may be null): max |x - xm|
hipError_t launch_filter(const Dev& d, const float* xm, const float* xp, const double* s_dev,
                         float* x, float* xm_out, unsigned long long* dxo, hipStream_t st);
// x = x^k at the end of an outer block without contact; dxo: max |x^k - x|
hipError_t launch_block_end(const Dev& d, unsigned long long* dxo, hipStream_t st);
// v = (x - x*) / h, or the rollback x = x* of a failed step (status in cnt)
hipError_t launch_epilogue(const Dev& d, float inv_h, int* cnt, hipStream_t st);
// clears the norm slots and the running step's status and counters
hipError_t launch_step_open(unsigned long long* dxbits, int nslots, int* cnt, int* gate, hipStream_t st);
// loop conditions of the tolerance mode (see k_gate)
hipError_t launch_gate(int* gate, const unsigned long long* dxbits, int prev_inner, double tol_in, int prev_outer,
                       double tol_out, int block, int* cnt, hipStream_t st);
// local step + residual r0 + U^T r0 partials (contact: W, WY read when has_contact)
// flags: bit 0 contact terms, bit 1 linear mode (b = 0), bit 2 obstacle weights k
hipError_t launch_local_residual(const Dev& d, int prec, int flags, hipStream_t st);
// sum of U^T r0 partials -> d.gvec; without contact also Q = A^{-1} g
hipError_t launch_reduce_solve(const Dev& d, int nblk, int contact, double* gpart2,
                               hipStream_t st);
// delta = U q into d.d4 (AoS); add: d.xt = x^k + U q (SoA)
hipError_t launch_expand(const Dev& d, int prec, int add, hipStream_t st);
// dx_prev (may be null): the slot a gated sweep repeats
// mode 0: Chebyshev blend; 1, 2: the two launches of a rank-2 A-Jacobi step
hipError_t launch_jacobi_cheb(const Dev& d, float omega, float gamma, int has_contact,
                              unsigned long long* dx_slot, const unsigned long long* dx_prev, hipStream_t st,
                              int mode = 0);

}  // namespace cloth
