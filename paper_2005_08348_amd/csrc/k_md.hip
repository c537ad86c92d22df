// k_md.hip -- Langevin BAOAB integration, steepest-descent steps, state
// import/export and small utility kernels.
#include "membx_dev.h"

namespace mbx {

// B (kick) + A + O + A of one BAOAB step, with the closing B of the previous
// step folded into `kick` (dt instead of dt/2 inside a run of steps), in
// place; x at the last rebuild is compared to flag displacements beyond
// skin/2.
template <typename R>
__global__ __launch_bounds__(WG) void k_kick_drift(Dev<R> d, R kick, long long step_off, int chk_in,
                                                   int bin)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    float e2 = 0.f, e2_in = 0.f;
    if (i < d.N)
        e2 = baoab_bead(d, i, d.posq[i], bead_pre(d, i, chk_in != 0), d.frc[i], kick, step_off,
                        d.posq, d.vel, chk_in != 0, e2_in);
    disp_stats(d, e2, e2_in, i < d.N);
    if (bin) {   // the rebuild that follows skips its binning
        int cell = -1;
        if (i < d.N) {
            V4<R> p = d.posq[i];   // this thread's own store above
            cell = bin_cell(d, p);
            d.posq[i] = p;
        }
        bin_place(d, i, cell);
    }
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

// The boundary between two MDAS segments (Eq. 3's increments, Langevin) in
// one pass, the operations of k_kick, k_work, k_dlam and k_kick_drift in
// that order: the closing half-kick of the last step at lambda, the work
// increment w += dlw dU (md[0], md[1]; thread 0), the affected beads'
// forces moved to the next lambda (F += dl (F_B - F_A)), and the opening
// B-A-O-A of the next segment's first step (step counter + step_off; the
// step counter itself advances at the cycle's last closing kick).
template <typename R>
__global__ __launch_bounds__(WG) void k_alch_bridge(Dev<R> d, const int* __restrict__ aff_flag,
                                                    double* md, R kick, R dl, double dlw,
                                                    long long step_off)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i == 0) md[0] += dlw * md[1];
    float e2 = 0.f, e2_in = 0.f;
    if (i < d.N) {
        BeadPre<R> pre = bead_pre(d, i, false);
        V4<R> f = d.frc[i];
        pre.v.x += kick * pre.v.w * f.x; pre.v.y += kick * pre.v.w * f.y;
        pre.v.z += kick * pre.v.w * f.z;
        if (aff_flag[i]) {
            const V4<R> g = d.dfrc[i];
            f.x += dl * g.x; f.y += dl * g.y; f.z += dl * g.z;
            d.frc[i] = f;
        }
        e2 = baoab_bead(d, i, d.posq[i], pre, f, kick, step_off, d.posq, d.vel, false, e2_in);
    }
    disp_stats(d, e2, e2_in, i < d.N);
}

// The same boundary on the soft-core path (Langevin): the operations of
// k_kick, k_work (weight 1: the work increment is U_sc(lam') - U_sc(lam)),
// k_scforce's update of the affected beads' forces (held in dsc in float64)
// and k_kick_drift in that order.
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_bridge(Dev<R> d, const int* __restrict__ aff_flag,
                                                 const double* __restrict__ dsc, double* md, R kick,
                                                 long long step_off)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i == 0) md[0] += 1.0 * md[1];
    float e2 = 0.f, e2_in = 0.f;
    if (i < d.N) {
        BeadPre<R> pre = bead_pre(d, i, false);
        V4<R> f = d.frc[i];
        pre.v.x += kick * pre.v.w * f.x; pre.v.y += kick * pre.v.w * f.y;
        pre.v.z += kick * pre.v.w * f.z;
        if (aff_flag[i]) {
            const double* g = dsc + 4 * (size_t)i;
            f.x = (R)((double)f.x + g[0]); f.y = (R)((double)f.y + g[1]); f.z = (R)((double)f.z + g[2]);
            d.frc[i] = f;
        }
        e2 = baoab_bead(d, i, d.posq[i], pre, f, kick, step_off, d.posq, d.vel, false, e2_in);
    }
    disp_stats(d, e2, e2_in, i < d.N);
}

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
void launch_kick_drift(const Dev<R>& d, R kick, long long step_off, int chk_in, hipStream_t st,
                       int bin)
{
    hipLaunchKernelGGL(k_kick_drift<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, kick,
                       step_off, chk_in, bin);
}
template <typename R>
void launch_sc_bridge(const Dev<R>& d, const int* aff_flag, const double* dsc, double* md, R kick,
                      long long step_off, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_bridge<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, aff_flag, dsc,
                       md, kick, step_off);
}
template <typename R>
void launch_alch_bridge(const Dev<R>& d, const int* aff_flag, double* md, R kick, R dl, double dlw,
                        long long step_off, hipStream_t st)
{
    hipLaunchKernelGGL(k_alch_bridge<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, aff_flag, md,
                       kick, dl, dlw, step_off);
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

// ------------------------------------------- stochastic velocity rescaling
// The paper's ensemble (Methods) keeps the temperature with the velocity
// rescaling thermostat of Bussi, Donadio and Parrinello (J. Chem. Phys. 126,
// 014101, 2007).  After the closing half-kick of each velocity Verlet step,
// the kinetic energy K of each coupling group (Nf = 3 x its beads) takes one
// exact step of that method's stochastic dynamics, c = exp(-dt / tau_t),
// Kt = Nf kT / 2:
//   K' = c K + (1 - c) Kt (R1^2 + S) / Nf + 2 R1 sqrt(c (1 - c) K Kt / Nf),
// R1 standard normal and S chi-squared with Nf - 1 degrees of freedom (twice a
// Gamma((Nf - 1) / 2) variate, Marsaglia-Tsang); the group's velocities are
// multiplied by alpha = sqrt(K' / K), with the sign of the new velocity
// component along the old one, R1 + sqrt(c Nf K / ((1 - c) Kt)).  Random
// words: Philox stream 5, counter = step index, block (group << 16) for R1
// and (group << 16) + 1 + t for the t-th attempt of the gamma sampler.  The
// half-kick with per-block group sums runs in the force pass itself (k_nb,
// FUSE 2) or, after an MDAS segment's alchemical forces, in k_kick_ke; every
// work-group of the next step's update (or of k_vr_scale after the last
// step) sums those partials and draws the two factors itself (float64
// throughout; all draw the same), then scales its beads' velocities.

template <typename R>
__global__ __launch_bounds__(WG) void k_kick_ke(Dev<R> d, VrBuf vr, R kick)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    double q[4] = { 0.0, 0.0, 0.0, 0.0 };   // K of group 0, 1; beads of group 0, 1
    if (i < d.N) {
        V4<R> v = d.vel[i];
        const V4<R> f = d.frc[i];
        v.x += kick * v.w * f.x; v.y += kick * v.w * f.y; v.z += kick * v.w * f.z;
        d.vel[i] = v;
        const double ek =
            0.5 * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z) / (double)v.w;
        const bool g1 = vr_group(d, vr, i) != 0;
        q[0] = g1 ? 0.0 : ek; q[1] = g1 ? ek : 0.0;
        q[2] = g1 ? 0.0 : 1.0; q[3] = g1 ? 1.0 : 0.0;
    }
    __shared__ double sw[4][WG / 64];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double x = q[c];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0) sw[c][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < WG / 64; ++w) t += sw[threadIdx.x][w];
        vr.part[4 * blockIdx.x + threadIdx.x] = t;
    }
}

// one standard normal from two words (Box-Muller, cosine branch)
__device__ __forceinline__ double vr_normal(uint32_t a, uint32_t b)
{
    const double s32 = 1.0 / 4294967296.0, tp = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(((double)a + 1.0) * s32)) * cos(tp * ((double)b * s32));
}

// Gamma(a, 1), a >= 1 (Marsaglia and Tsang, ACM TOMS 26, 363, 2000), at most
// 64 attempts
__device__ double vr_gamma(uint64_t seed, int g, double a, long long ctr)
{
    const double dd = a - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * dd);
    for (int t = 0; t < 64; ++t) {
        const uint4 w = draw(seed, (uint32_t)((g << 16) + 1 + t), ctr, ST_VRESCALE);
        const double x = vr_normal(w.x, w.y), u = u53(w.z, w.w);
        const double y = 1.0 + cc * x;
        if (y <= 0.0) continue;
        const double v = y * y * y;
        if (log(u) < 0.5 * x * x + dd - dd * v + dd * log(v)) return dd * v;
    }
    return dd;
}

__device__ double vr_factor(uint64_t seed, int g, double K, double nf, double kT, double c,
                            long long ctr)
{
    if (!(K > 0.0) || !(nf >= 3.0)) return 1.0;
    const double kt = 0.5 * nf * kT;
    const uint4 w = draw(seed, (uint32_t)(g << 16), ctr, ST_VRESCALE);
    const double r1 = vr_normal(w.x, w.y);
    const double sch = 2.0 * vr_gamma(seed, g, 0.5 * (nf - 1.0), ctr);
    const double kn = K + (1.0 - c) * (kt * (r1 * r1 + sch) / nf - K) +
                      2.0 * r1 * sqrt(c * (1.0 - c) * K * kt / nf);
    const double al = sqrt(kn / K);
    return (r1 + sqrt(c * nf * K / ((1.0 - c) * kt)) < 0.0) ? -al : al;
}

// The step's two factors from the nblk block partials of its closing
// half-kick: sums in a fixed order (strided over the work-group's threads,
// then its waves), then threads 0 and 1 draw the factors of groups 0 and 1
// into al (LDS).  Every thread of the work-group calls it; each work-group
// of the update that applies the factors runs it itself, so no separate
// launch waits between the force pass and the update.
template <typename R>
__device__ __forceinline__ void vr_factors_wg(const Dev<R>& d, const VrBuf& vr, int nblk,
                                              long long fstep, double c, double* al)
{
    const int t = threadIdx.x;
    double q[4] = { 0.0, 0.0, 0.0, 0.0 };
    for (int b = t; b < nblk; b += WG)
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] += vr.part[4 * b + k];
    __shared__ double sw[4][WG / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        for (int o = 32; o > 0; o >>= 1) q[k] += __shfl_xor(q[k], o, 64);
        if ((t & 63) == 0) sw[k][t >> 6] = q[k];
    }
    __syncthreads();
    if (t < 2) {
        double K = 0.0, nb = 0.0;
        for (int w = 0; w < WG / 64; ++w) { K += sw[t][w]; nb += sw[2 + t][w]; }
        al[t] = vr_factor(d.seed, t, K, 3.0 * nb, d.kTd, c, d.ctr[CT_STEP] + fstep);
        if (blockIdx.x == 0) vr.alpha[t] = al[t];   // the last factors, for the record
    }
    __syncthreads();
}

// the last step's factors applied after a sequence of steps
template <typename R>
__global__ __launch_bounds__(WG) void k_vr_scale(Dev<R> d, VrBuf vr, int nblk, long long fstep,
                                                 double c)
{
    __shared__ double al[2];
    vr_factors_wg(d, vr, nblk, fstep, c, al);
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    const double a = al[vr_group(d, vr, i)];
    V4<R> v = d.vel[i];
    v.x = (R)(a * (double)v.x); v.y = (R)(a * (double)v.y); v.z = (R)(a * (double)v.z);
    d.vel[i] = v;
}

// ------------------------------------------------- pressure coupling
// Semi-isotropic stochastic cell rescaling (the paper's 1 bar barostat,
// Methods; Bernetti and Bussi 2020): the log-strains e_A = ln(Lx Ly) and
// e_z = ln Lz each take one Ito Euler-Maruyama step over t,
//   d e = -(kappa / tau_p) (P0 - P) t + sqrt(2 kappa kT t / (V tau_p)) xi,
// P_A = (N kT + (W_xx + W_yy) / 2) / V, P_z = (N kT + W_zz) / V, from the
// virial of the energy pass (eout[7..9]); xi from Philox stream 6, block 0,
// counter = the step index.  One thread writes the scale factors
// {exp(d e_A / 2), exp(d e_A / 2), exp(d e_z)} to mu[0..2].
template <typename R>
__global__ void k_baro(Dev<R> d, const double* __restrict__ eout, double* __restrict__ mu,
                       double p0, double kappa, double tau_p, double t, double vol)
{
    if (threadIdx.x != 0) return;
    const double nkt = (double)d.N * d.kTd;
    const double pa = (nkt + 0.5 * (eout[7] + eout[8])) / vol, pz = (nkt + eout[9]) / vol;
    const uint4 w = draw(d.seed, 0u, d.ctr[CT_STEP], ST_BARO);
    const double xa = vr_normal(w.x, w.y), xz = vr_normal(w.z, w.w);
    const double drift = kappa / tau_p * t, amp = sqrt(2.0 * kappa * d.kTd * t / (vol * tau_p));
    const double dea = -drift * (p0 - pa) + amp * xa;
    const double dez = -drift * (p0 - pz) + amp * xz;
    mu[0] = exp(0.5 * dea);
    mu[1] = exp(0.5 * dea);
    mu[2] = exp(dez);
}

// positions scaled about the origin (slots; the rebuild that follows wraps
// them and places the images)
template <typename R>
__global__ __launch_bounds__(WG) void k_scale_pos(Dev<R> d, double mx, double my, double mz)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    V4<R> p = d.posq[i];
    p.x = (R)(mx * (double)p.x); p.y = (R)(my * (double)p.y); p.z = (R)(mz * (double)p.z);
    d.posq[i] = p;
}

// peculiar velocities divided by the box stretch per axis (a Parrinello-
// Rahman box move at fixed scaled coordinates and their momenta)
template <typename R>
__global__ __launch_bounds__(WG) void k_unscale_vel(Dev<R> d, double mx, double my, double mz)
{
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.N) return;
    V4<R> v = d.vel[i];
    v.x = (R)((double)v.x / mx); v.y = (R)((double)v.y / my); v.z = (R)((double)v.z / mz);
    d.vel[i] = v;
}

template <typename R>
void launch_unscale_vel(const Dev<R>& d, const double* mu, hipStream_t st)
{
    hipLaunchKernelGGL(k_unscale_vel<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, mu[0], mu[1],
                       mu[2]);
}

template <typename R>
void launch_baro(const Dev<R>& d, const double* eout, double* mu, double p0, double kappa,
                 double tau_p, double t, double vol, hipStream_t st)
{
    hipLaunchKernelGGL(k_baro<R>, dim3(1), dim3(64), 0, st, d, eout, mu, p0, kappa, tau_p, t, vol);
}
template <typename R>
void launch_scale_pos(const Dev<R>& d, const double* mu, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_pos<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, mu[0], mu[1],
                       mu[2]);
}

// the previous step's scaling folded into this step's B-A-O-A (the O part is
// off under this thermostat): v <- alpha_g v, then the kick and drifts; the
// factors come from that step's nblk block partials (counter: step fstep)
template <typename R>
__global__ __launch_bounds__(WG) void k_vr_kick_drift(Dev<R> d, VrBuf vr, R kick, long long step_off,
                                                      int chk_in, int nblk, long long fstep, double c,
                                                      int bin)
{
    __shared__ double al[2];
    vr_factors_wg(d, vr, nblk, fstep, c, al);
    const int i = blockIdx.x * WG + threadIdx.x;
    float e2 = 0.f, e2_in = 0.f;
    if (i < d.N) {
        BeadPre<R> pre = bead_pre(d, i, chk_in != 0);
        const double a = al[vr_group(d, vr, i)];
        pre.v.x = (R)(a * (double)pre.v.x);
        pre.v.y = (R)(a * (double)pre.v.y);
        pre.v.z = (R)(a * (double)pre.v.z);
        e2 = baoab_bead(d, i, d.posq[i], pre, d.frc[i], kick, step_off, d.posq, d.vel, chk_in != 0,
                        e2_in);
    }
    disp_stats(d, e2, e2_in, i < d.N);
    if (bin) {   // the rebuild that follows skips its binning
        int cell = -1;
        if (i < d.N) {
            V4<R> p = d.posq[i];   // this thread's own store above
            cell = bin_cell(d, p);
            d.posq[i] = p;
        }
        bin_place(d, i, cell);
    }
}

// closing half-kick with the group sums (after an MDAS segment's alchemical
// forces; otherwise the force pass makes it, FUSE 2); returns the number of
// block partials.  The factors are drawn where they are applied
// (k_vr_kick_drift of the next step, or k_vr_scale after the last).
template <typename R>
int launch_kick_ke(const Dev<R>& d, const VrBuf& vr, R kick, hipStream_t st)
{
    const int nb = (d.N + WG - 1) / WG;
    hipLaunchKernelGGL(k_kick_ke<R>, dim3(nb), dim3(WG), 0, st, d, vr, kick);
    return nb;
}
template <typename R>
void launch_vr_scale(const Dev<R>& d, const VrBuf& vr, int nblk, long long fstep, double c,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_vr_scale<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, vr, nblk, fstep,
                       c);
}
template <typename R>
void launch_vr_kick_drift(const Dev<R>& d, const VrBuf& vr, R kick, long long step_off, int chk_in,
                          int nblk, long long fstep, double c, hipStream_t st, int bin)
{
    hipLaunchKernelGGL(k_vr_kick_drift<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, vr, kick,
                       step_off, chk_in, nblk, fstep, c, bin);
}

#define INST(R)                                                                      \
    template int launch_kick_ke<R>(const Dev<R>&, const VrBuf&, R, hipStream_t);     \
    template void launch_vr_scale<R>(const Dev<R>&, const VrBuf&, int, long long, double, \
                                     hipStream_t);                                   \
    template void launch_baro<R>(const Dev<R>&, const double*, double*, double, double, double, \
                                 double, double, hipStream_t);                       \
    template void launch_scale_pos<R>(const Dev<R>&, const double*, hipStream_t);    \
    template void launch_unscale_vel<R>(const Dev<R>&, const double*, hipStream_t);  \
    template void launch_vr_kick_drift<R>(const Dev<R>&, const VrBuf&, R, long long, int, int, \
                                          long long, double, hipStream_t, int);      \
    template void launch_kick_drift<R>(const Dev<R>&, R, long long, int, hipStream_t, int); \
    template void launch_kick<R>(const Dev<R>&, R, long long, hipStream_t);                    \
    template void launch_sc_bridge<R>(const Dev<R>&, const int*, const double*, double*, R,      \
                                      long long, hipStream_t);                                 \
    template void launch_alch_bridge<R>(const Dev<R>&, const int*, double*, R, R, double, long long, \
                                        hipStream_t);                                          \
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
