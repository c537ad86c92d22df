// k_md.hip -- Langevin BAOAB integration, steepest-descent steps, state
// import/export and small utility kernels.
#include "membx_dev.h"

namespace mbx {

// B (kick) + A + O + A of one BAOAB step, with the closing B of the previous
// step folded into `kick` (dt instead of dt/2 inside a run of steps), in
// place; x at the last rebuild is compared to flag displacements beyond
// skin/2.
template <typename R>
__global__ __launch_bounds__(WG) void k_kick_drift(Dev<R> d, R kick, long long step_off, int chk_in)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    float e2 = 0.f, e2_in = 0.f;
    if (i < d.N)
        e2 = baoab_bead(d, i, d.posq[i], bead_pre(d, i, chk_in != 0), d.frc[i], kick, step_off,
                        d.posq, d.vel, chk_in != 0, e2_in);
    disp_stats(d, e2, e2_in, i < d.N);
}

// closing half-kick of a run of steps; also advances the step counter
template <typename R>
__global__ __launch_bounds__(WG) void k_kick(Dev<R> d, R kick, long long nsteps)
{
    int i = blockIdx.x * WG + threadIdx.x;
    if (i == 0 && nsteps) d.ctr[CT_STEP] += nsteps;
    if (i >= d.N) return;
    V4<R> v = d.vel[i], f = d.frc[i];
    v.x += kick * v.w * f.x; v.y += kick * v.w * f.y; v.z += kick * v.w * f.z;
    d.vel[i] = v;
}

__global__ void k_add_ctr(long long* ctr, int which, long long n) { ctr[which] += n; }

// capped steepest-descent step: x += s * alpha F, |s alpha F| <= cap
template <typename R>
__global__ void k_sd_step(Dev<R> d, double alpha, double cap)
{
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    V4<R> p = d.posq[i], f = d.frc[i];
    double dx = alpha * (double)f.x, dy = alpha * (double)f.y, dz = alpha * (double)f.z;
    double l = sqrt(dx * dx + dy * dy + dz * dz);
    double sc = l > cap ? cap / l : 1.0;
    if (!(l == l)) sc = 0.0;
    p.x = (R)((double)p.x + sc * dx);
    p.y = (R)((double)p.y + sc * dy);
    p.z = (R)((double)p.z + sc * dz);
    d.posq[i] = p;
}

// export in bead-id order as float64 triples
template <typename R>
__global__ void k_export(Dev<R> d, const V4<R>* __restrict__ src, double* __restrict__ out)
{
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    V4<R> v = src[i];
    int o = d.orig[i];
    out[3 * o] = (double)v.x; out[3 * o + 1] = (double)v.y; out[3 * o + 2] = (double)v.z;
}

// import float64 triples in bead-id order into slots (w kept)
template <typename R>
__global__ void k_import(Dev<R> d, V4<R>* dst, const double* __restrict__ in)
{
    int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    int o = d.orig[i];
    V4<R> v = dst[i];
    v.x = (R)in[3 * o]; v.y = (R)in[3 * o + 1]; v.z = (R)in[3 * o + 2];
    dst[i] = v;
}

__global__ void k_fill_i32(int* p, int v, size_t n)
{
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n)
{
    size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    size_t stride = (size_t)gridDim.x * WG;
    for (; i < n; i += stride) dst[i] = src[i];
}

void launch_fill_i32(int* p, int v, size_t n, hipStream_t st)
{
    if (!n) return;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st, p, v, n);
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    size_t n = bytes / 16;
    if (!n) return;
    size_t blocks = (n + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(WG), 0, st, (uint4*)dst,
                       (const uint4*)src, n);
}

void launch_add_ctr(long long* ctr, int which, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_ctr, dim3(1), dim3(1), 0, st, ctr, which, n);
}

template <typename R>
void launch_kick_drift(const Dev<R>& d, R kick, long long step_off, int chk_in, hipStream_t st)
{
    hipLaunchKernelGGL(k_kick_drift<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, kick,
                       step_off, chk_in);
}
template <typename R>
void launch_kick(const Dev<R>& d, R kick, long long nsteps, hipStream_t st)
{
    hipLaunchKernelGGL(k_kick<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, kick, nsteps);
}
template <typename R>
void launch_sd_step(const Dev<R>& d, double alpha, double cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_sd_step<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, alpha, cap);
}
template <typename R>
void launch_export(const Dev<R>& d, const V4<R>* src, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_export<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, src, out);
}
template <typename R>
void launch_import(const Dev<R>& d, V4<R>* dst, const double* in, hipStream_t st)
{
    hipLaunchKernelGGL(k_import<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, dst, in);
}

#define INST(R)                                                                      \
    template void launch_kick_drift<R>(const Dev<R>&, R, long long, int, hipStream_t); \
    template void launch_kick<R>(const Dev<R>&, R, long long, hipStream_t);                    \
    template void launch_sd_step<R>(const Dev<R>&, double, double, hipStream_t);     \
    template void launch_export<R>(const Dev<R>&, const V4<R>*, double*, hipStream_t); \
    template void launch_import<R>(const Dev<R>&, V4<R>*, const double*, hipStream_t);
INST(float)
INST(double)

}  // namespace mbx

namespace mbx {
// set every slot's class from a per-bead table (after a change of kinds)
template <typename R>
__global__ void k_set_classes(V4<R>* posq, const int* __restrict__ cls, const int* __restrict__ orig,
                              int N)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s >= N) return;
    V4<R> p = posq[s];
    p.w = cls_to<R>(cls[orig[s]]);
    posq[s] = p;
}

void launch_set_classes(void* posq, int prec, const int* cls, const int* orig, int N, hipStream_t st)
{
    dim3 g((N + WG - 1) / WG);
    if (prec == 1) hipLaunchKernelGGL(k_set_classes<float>, g, dim3(WG), 0, st, (V4<float>*)posq, cls, orig, N);
    else hipLaunchKernelGGL(k_set_classes<double>, g, dim3(WG), 0, st, (V4<double>*)posq, cls, orig, N);
}
}  // namespace mbx
