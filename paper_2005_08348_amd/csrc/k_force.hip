// k_force.hip -- nonbonded pair forces (potential-shifted LJ 12-6 + reaction
// field, paper Methods), bonded forces (harmonic bonds, cos^2 angles), kinetic
// energy and the deterministic float64 energy reduction.
//
// Nonbonded kernel.  Pair forces are not a dense contraction, so the kernel
// runs on the vector ALUs: LPB lanes of a wave64 share one i bead and walk
// its full (both-direction) Verlet list in an interleaved order; the j bead's
// coordinates and class come in one 16-byte gather, the pair parameters from
// a class-by-class table in LDS.  Each i force is the in-register sum over its
// list followed by a fixed shuffle tree over its LPB lanes, so results are
// deterministic and no atomics are used.
#include "membx_dev.h"

namespace mbx {

template <typename R> __device__ __forceinline__ R rsq(R x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

template <typename R, bool EN>
__device__ __forceinline__ void pair_force(const Dev<R>& d, const V4<R>* __restrict__ rowF,
                                           const V4<R>* __restrict__ rowE, R dx, R dy, R dz,
                                           R wj, R& fx, R& fy, R& fz, double& elj,
                                           double& erf, int& np)
{
    R r2 = dx * dx + dy * dy + dz * dz;
    int cj = cls_of<R>(wj);
    V4<R> p = rowF[cj];
    R rinv = rsq<R>(r2);
    R rinv2 = rinv * rinv;
    R rinv6 = rinv2 * rinv2 * rinv2;
    R fs = (p.y * rinv6 - p.x) * (rinv6 * rinv2) + (p.z * (rinv * rinv2) - p.w);
    bool in = r2 < d.rc2;
    fs = in ? fs : (R)0;
    fx += fs * dx;
    fy += fs * dy;
    fz += fs * dz;
    if (EN) {
        V4<R> q = rowE[cj];
        R vlj = (q.y * rinv6 - q.x) * rinv6 - q.w;
        R vrf = q.z * (rinv + d.krf * r2 - d.crf);
        if (in) {
            elj += (double)vlj;
            erf += (double)vrf;
            np += 1;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// block (WG threads) sum of three doubles into red[slot*4 + 0..2]; thread 0 writes
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* out)
{
    __shared__ double sh[3][WG / 64];
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { s0 += sh[0][q]; s1 += sh[1][q]; s2 += sh[2][q]; }
        out[0] = s0; out[1] = s1; out[2] = s2; out[3] = 0.0;
    }
}

template <typename R, int LPB, bool EN>
__global__ __launch_bounds__(WG) void k_nb(Dev<R> d, double* __restrict__ part)
{
    __shared__ V4<R> tf[MAXCLS * MAXCLS];
    __shared__ V4<R> te[EN ? MAXCLS * MAXCLS : 1];
    for (int t = threadIdx.x; t < MAXCLS * MAXCLS; t += WG) {
        tf[t] = d.tabF[t];
        if (EN) te[t] = d.tabE[t];
    }
    __syncthreads();
    const int gid = blockIdx.x * WG + threadIdx.x;
    const int i = gid / LPB, s = gid % LPB;
    const bool valid = i < d.N;
    V4<R> pi = valid ? d.posq[i] : V4<R>{ 0, 0, 0, 0 };
    const int ci = valid ? cls_of<R>(pi.w) : 0;
    const int n0 = valid ? d.nseg0[i] : 0, n1 = valid ? d.ncnt[i] : 0;
    const V4<R>* rowF = tf + ci * MAXCLS;
    const V4<R>* rowE = EN ? te + ci * MAXCLS : tf;
    R fx = 0, fy = 0, fz = 0;
    double elj = 0.0, erf = 0.0;
    int np = 0;
    const int* __restrict__ nb = d.nbr + (valid ? i : 0);
    const size_t stride = (size_t)d.Npad;
    for (int k = s; k < n0; k += LPB) {
        int j = nb[(size_t)k * stride];
        V4<R> pj = d.posq[j];
        pair_force<R, EN>(d, rowF, rowE, pi.x - pj.x, pi.y - pj.y, pi.z - pj.z, pj.w, fx, fy,
                          fz, elj, erf, np);
    }
    for (int k = n0 + s; k < n1; k += LPB) {
        int e = nb[(size_t)k * stride];
        int j = e & JMASK, code = (int)((unsigned)e >> CODE_SHIFT);
        V4<R> pj = d.posq[j];
        R xs = (code & 1) ? pi.x - d.L[0] : pi.x;
        R ys = (code & 2) ? pi.y - d.L[1] : pi.y;
        R zs = (code & 4) ? pi.z - d.L[2] : pi.z;
        pair_force<R, EN>(d, rowF, rowE, xs - pj.x, ys - pj.y, zs - pj.z, pj.w, fx, fy, fz, elj,
                          erf, np);
    }
#pragma unroll
    for (int m = LPB / 2; m >= 1; m >>= 1) {
        fx += __shfl_xor(fx, m);
        fy += __shfl_xor(fy, m);
        fz += __shfl_xor(fz, m);
    }
    if (!EN) {
        if (valid && s == 0) d.frc[i] = V4<R>{ fx, fy, fz, (R)0 };
    } else {
        block_sum3(elj, erf, (double)np, part + 4 * blockIdx.x);
    }
}

// Exact minimum-image separation for bonded partners: the coordinate near
// the top face is shifted down by L first (exact since it is >= L/2).
template <typename R>
__device__ __forceinline__ R sep(R xi, R xj, R L, R hL)
{
    R dx = xi - xj;
    if (dx > hL) dx = (xi - L) - xj;
    else if (dx < -hL) dx = xi - (xj - L);
    return dx;
}

template <typename R, bool EN>
__global__ __launch_bounds__(64) void k_bonded(Dev<R> d, double* __restrict__ part)
{
    __shared__ R fl[64][MAXMB * 3];
    __shared__ V4<R> pl[64][MAXMB];
    __shared__ int sl[64][MAXMB];
    const int t = blockIdx.x * 64 + threadIdx.x;
    double eb = 0.0, ea = 0.0;
    if (t < d.nbm) {
        const int m = d.bmols[t], k = d.mol_kind[m], f0 = d.mol_first[m], nb = d.kn[k];
        R* f = fl[threadIdx.x];
        V4<R>* p = pl[threadIdx.x];
        int* sv = sl[threadIdx.x];
        for (int b = 0; b < nb; ++b) {
            int s = d.inv[f0 + b];
            sv[b] = s;
            p[b] = d.posq[s];
            f[3 * b] = f[3 * b + 1] = f[3 * b + 2] = (R)0;
        }
        const int q0 = d.kb_off[k], qn = d.kb_n[k];
        for (int q = q0; q < q0 + qn; ++q) {
            int li = d.b_ij[2 * q], lj = d.b_ij[2 * q + 1];
            R b0 = d.b_par[2 * q], kb = d.b_par[2 * q + 1];
            R dx = sep(p[li].x, p[lj].x, d.L[0], d.halfL[0]);
            R dy = sep(p[li].y, p[lj].y, d.L[1], d.halfL[1]);
            R dz = sep(p[li].z, p[lj].z, d.L[2], d.halfL[2]);
            R r = sqrt(dx * dx + dy * dy + dz * dz);
            R dr = r - b0;
            R fs = -kb * dr / r;
            f[3 * li] += fs * dx; f[3 * li + 1] += fs * dy; f[3 * li + 2] += fs * dz;
            f[3 * lj] -= fs * dx; f[3 * lj + 1] -= fs * dy; f[3 * lj + 2] -= fs * dz;
            if (EN) eb += 0.5 * (double)kb * (double)dr * (double)dr;
        }
        const int a0 = d.ka_off[k], an = d.ka_n[k];
        for (int q = a0; q < a0 + an; ++q) {
            int li = d.a_ijk[3 * q], lj = d.a_ijk[3 * q + 1], lk = d.a_ijk[3 * q + 2];
            R c0 = d.a_par[2 * q], ka = d.a_par[2 * q + 1];
            R ux = sep(p[li].x, p[lj].x, d.L[0], d.halfL[0]);
            R uy = sep(p[li].y, p[lj].y, d.L[1], d.halfL[1]);
            R uz = sep(p[li].z, p[lj].z, d.L[2], d.halfL[2]);
            R wx = sep(p[lk].x, p[lj].x, d.L[0], d.halfL[0]);
            R wy = sep(p[lk].y, p[lj].y, d.L[1], d.halfL[1]);
            R wz = sep(p[lk].z, p[lj].z, d.L[2], d.halfL[2]);
            R uu = ux * ux + uy * uy + uz * uz, ww = wx * wx + wy * wy + wz * wz;
            R inw = (R)1 / sqrt(uu * ww);
            R c = (ux * wx + uy * wy + uz * wz) * inw;
            R dc = c - c0;
            R pre = -ka * dc;
            R cu = c / uu, cw = c / ww;
            R dix = wx * inw - cu * ux, diy = wy * inw - cu * uy, diz = wz * inw - cu * uz;
            R dkx = ux * inw - cw * wx, dky = uy * inw - cw * wy, dkz = uz * inw - cw * wz;
            f[3 * li] += pre * dix; f[3 * li + 1] += pre * diy; f[3 * li + 2] += pre * diz;
            f[3 * lk] += pre * dkx; f[3 * lk + 1] += pre * dky; f[3 * lk + 2] += pre * dkz;
            f[3 * lj] -= pre * (dix + dkx);
            f[3 * lj + 1] -= pre * (diy + dky);
            f[3 * lj + 2] -= pre * (diz + dkz);
            if (EN) ea += 0.5 * (double)ka * (double)dc * (double)dc;
        }
        if (!EN) {
            for (int b = 0; b < nb; ++b) {
                V4<R> g = d.frc[sv[b]];
                g.x += f[3 * b]; g.y += f[3 * b + 1]; g.z += f[3 * b + 2];
                d.frc[sv[b]] = g;
            }
        }
    }
    if (EN) {
        eb = wave_sum(eb);
        ea = wave_sum(ea);
        if (threadIdx.x == 0) { part[4 * blockIdx.x] = eb; part[4 * blockIdx.x + 1] = ea; }
    }
}

template <typename R>
__global__ __launch_bounds__(WG) void k_kinetic(Dev<R> d, double* __restrict__ part)
{
    int i = blockIdx.x * WG + threadIdx.x;
    double ke = 0.0;
    if (i < d.N) {
        V4<R> v = d.vel[i];
        double v2 = (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z;
        ke = 0.5 * v2 / (double)v.w;
    }
    block_sum3(ke, 0.0, 0.0, part + 4 * blockIdx.x);
}

// Fixed-order float64 sum of the block partials:
// out = {lj, rf, bond, angle, kinetic, n_pairs}
__global__ void k_energy_final(const double* __restrict__ pnb, int nnb,
                               const double* __restrict__ pbd, int nbd,
                               const double* __restrict__ pke, int nke, double* __restrict__ out)
{
    __shared__ double sh[6][256];
    int t = threadIdx.x;
    double a[6] = { 0, 0, 0, 0, 0, 0 };
    for (int b = t; b < nnb; b += 256) { a[0] += pnb[4 * b]; a[1] += pnb[4 * b + 1]; a[5] += pnb[4 * b + 2]; }
    for (int b = t; b < nbd; b += 256) { a[2] += pbd[4 * b]; a[3] += pbd[4 * b + 1]; }
    for (int b = t; b < nke; b += 256) { a[4] += pke[4 * b]; }
    for (int q = 0; q < 6; ++q) sh[q][t] = a[q];
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (t < off)
            for (int q = 0; q < 6; ++q) sh[q][t] += sh[q][t + off];
        __syncthreads();
    }
    if (t == 0) {
        // every unordered pair appears twice in the full lists
        out[0] = 0.5 * sh[0][0];
        out[1] = 0.5 * sh[1][0];
        out[2] = sh[2][0];
        out[3] = sh[3][0];
        out[4] = sh[4][0];
        out[5] = 0.5 * sh[5][0];
    }
}

// ----------------------------------------------------------------- launch
template <typename R, int LPB, bool EN>
static void nb_launch(const Dev<R>& d, double* part, hipStream_t st)
{
    int nthr = d.N * LPB;
    hipLaunchKernelGGL((k_nb<R, LPB, EN>), dim3((nthr + WG - 1) / WG), dim3(WG), 0, st, d, part);
}

template <typename R>
int nb_blocks(const Dev<R>& d, int lpb) { return (d.N * lpb + WG - 1) / WG; }

template <typename R>
void launch_nonbonded(const Dev<R>& d, int lpb, bool energy, double* part, hipStream_t st)
{
    switch (lpb * 2 + (energy ? 1 : 0)) {
    case 2: nb_launch<R, 1, false>(d, part, st); break;
    case 3: nb_launch<R, 1, true>(d, part, st); break;
    case 4: nb_launch<R, 2, false>(d, part, st); break;
    case 5: nb_launch<R, 2, true>(d, part, st); break;
    case 8: nb_launch<R, 4, false>(d, part, st); break;
    case 9: nb_launch<R, 4, true>(d, part, st); break;
    case 16: nb_launch<R, 8, false>(d, part, st); break;
    case 17: nb_launch<R, 8, true>(d, part, st); break;
    default: break;
    }
}

template <typename R>
void launch_bonded(const Dev<R>& d, bool energy, double* part, hipStream_t st)
{
    if (d.nbm == 0) return;
    dim3 g((d.nbm + 63) / 64);
    if (energy) hipLaunchKernelGGL((k_bonded<R, true>), g, dim3(64), 0, st, d, part);
    else hipLaunchKernelGGL((k_bonded<R, false>), g, dim3(64), 0, st, d, part);
}

template <typename R>
void launch_kinetic(const Dev<R>& d, double* part, hipStream_t st)
{
    hipLaunchKernelGGL(k_kinetic<R>, dim3((d.N + WG - 1) / WG), dim3(WG), 0, st, d, part);
}

void launch_energy_final(const double* pnb, int nnb, const double* pbd, int nbd,
                         const double* pke, int nke, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, st, pnb, nnb, pbd, nbd, pke, nke,
                       out);
}

template void launch_nonbonded<float>(const Dev<float>&, int, bool, double*, hipStream_t);
template void launch_nonbonded<double>(const Dev<double>&, int, bool, double*, hipStream_t);
template void launch_bonded<float>(const Dev<float>&, bool, double*, hipStream_t);
template void launch_bonded<double>(const Dev<double>&, bool, double*, hipStream_t);
template void launch_kinetic<float>(const Dev<float>&, double*, hipStream_t);
template void launch_kinetic<double>(const Dev<double>&, double*, hipStream_t);

}  // namespace mbx
