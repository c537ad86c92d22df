// k_force.hip -- forces and energies: nonbonded pair terms (potential-shifted
// LJ 12-6 + reaction field, paper Methods) and the Martini bonded terms
// (harmonic bonds, cos^2 angles), in one kernel, plus the deterministic
// float64 energy reduction.
//
// Pair forces are not a dense contraction, so the kernel runs on the vector
// ALUs: LPB lanes of a wave64 share one i bead and walk its full
// (both-direction) Verlet list.  The kernel is organised around memory
// latency and occupancy: per batch a lane issues its list reads (one
// contiguous 256-byte block per wave each, the list is tiled), then all the
// batch's coordinate gathers, then computes the batch without branches;
// registers are kept few (reads needed only after the walk are issued after
// it) so that more waves hide the latency.
// The j bead's coordinates and class come in one 16-byte gather and the pair
// parameters from a class-by-class table in LDS.  The same lanes then
// evaluate the bonded terms their bead takes part in (per-bead gather, no
// atomics).  Each force is an in-register sum followed by a fixed shuffle
// tree over the LPB lanes, so results are deterministic.
#include <type_traits>

#include "membx_dev.h"

namespace mbx {

template <typename R> __device__ __forceinline__ R rsq(R x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

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

template <typename R>
__device__ __forceinline__ void sep3(const Dev<R>& d, const V4<R>& a, const V4<R>& b, R& x, R& y,
                                     R& z)
{
    x = sep(a.x, b.x, d.L[0], d.halfL[0]);
    y = sep(a.y, b.y, d.L[1], d.halfL[1]);
    z = sep(a.z, b.z, d.L[2], d.halfL[2]);
}

// Force on bead i from one bonded term it takes part in (partner coordinates
// p1, p2 already gathered); energy and virial counted by the term's owner
// (bond role 0, angle vertex): for a bond (r_i - r_j)_a (F_i)_a, for an angle
// the ends' separations from the vertex times the ends' forces.
template <typename R, bool EN>
__device__ __forceinline__ void bonded_term(const Dev<R>& d, const V4<R>& pi, int4 tm,
                                            const V4<R>& p1, const V4<R>& p2, R& fx, R& fy, R& fz,
                                            double& eb, double& ea, double* wb)
{
    const R p0 = d.bt_par[2 * tm.w], kk = d.bt_par[2 * tm.w + 1];
    if (tm.x <= 1) {
        R dx, dy, dz;
        sep3(d, pi, p1, dx, dy, dz);
        R r = sqrt(dx * dx + dy * dy + dz * dz);
        R dr = r - p0;
        R fs = -kk * dr / r;
        fx += fs * dx; fy += fs * dy; fz += fs * dz;
        if (EN && tm.x == 0) {
            eb += 0.5 * (double)kk * (double)dr * (double)dr;
            wb[0] += (double)(fs * dx) * (double)dx;
            wb[1] += (double)(fs * dy) * (double)dy;
            wb[2] += (double)(fs * dz) * (double)dz;
        }
    } else {
        // role 2: i is an end, p1 the vertex, p2 the other end
        // role 3: i is the vertex, p1 and p2 the ends
        R ax, ay, az, bx, by, bz;
        if (tm.x == 2) { sep3(d, pi, p1, ax, ay, az); sep3(d, p2, p1, bx, by, bz); }
        else { sep3(d, p1, pi, ax, ay, az); sep3(d, p2, pi, bx, by, bz); }
        R aa = ax * ax + ay * ay + az * az, bb = bx * bx + by * by + bz * bz;
        R inw = (R)1 / sqrt(aa * bb);
        R c = (ax * bx + ay * by + az * bz) * inw;
        R dc = c - p0;
        R pre = -kk * dc;
        R ca = c / aa;
        R gx = bx * inw - ca * ax, gy = by * inw - ca * ay, gz = bz * inw - ca * az;  // dc/d(end a)
        if (tm.x == 2) {
            fx += pre * gx; fy += pre * gy; fz += pre * gz;
        } else {
            R cb = c / bb;
            R hx = ax * inw - cb * bx, hy = ay * inw - cb * by, hz = az * inw - cb * bz;
            fx -= pre * (gx + hx); fy -= pre * (gy + hy); fz -= pre * (gz + hz);
            if (EN) {
                ea += 0.5 * (double)kk * (double)dc * (double)dc;
                wb[0] += (double)ax * (double)(pre * gx) + (double)bx * (double)(pre * hx);
                wb[1] += (double)ay * (double)(pre * gy) + (double)by * (double)(pre * hy);
                wb[2] += (double)az * (double)(pre * gz) + (double)bz * (double)(pre * hz);
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// energies: partial[16 * block] = {lj, rf, pairs, bond, angle, kinetic,
// list entries, pair virial (3, both directions), bonded virial (3),
// m v_a^2 (3)}.
// FUSE 1: the lane that owns bead i's force also moves the bead through the
// next BAOAB step (its own force is all that step needs), writing the new
// coordinates to pos_out (the other coordinate buffer: the neighbours' old
// coordinates are still being read) and the velocity to vel_out.
// FUSE 2 (velocity rescaling): it makes the step's closing half-kick
// v += kick F / m instead and writes the block's kinetic energies and bead
// counts of the two coupling groups to part[4 * block .. + 3], the input of
// the thermostat's factors.
// LIST: 0 walk the Verlet list; 1 walk the inner list; 2 walk the Verlet
// list and rewrite the inner list from it (dynamic pruning): lane s of bead i
// keeps its entries within r_cut + delta, in order, as its own entries
// s, s + LPB, ... of the inner list, with its own count, and the bead's
// coordinates become the reference for the inner list's displacement check.
// stats: bit 0 the displacement bookkeeping; bit 1 (FUSE 1) the binning of
// the list build that follows (k_bin's work, on the new coordinates).
// FUSE 3 (MDAS segment boundary, in place of the closing pass of a segment
// and the next one's opening update): as FUSE 1, but the integrating thread
// first adds lam (F_B - F_A) to an affected bead's force, makes the closing
// half-kick with it, moves the force to lam + dl and makes the opening
// B-A-O-A with that (kick = dt / 2); one thread adds the work increment
// dlw dU.  The operations and their order are those of the separate passes.
template <typename R, int LPB, bool EN, int FUSE, int LIST>
__global__ __launch_bounds__(WG) void k_nb(Dev<R> d, double* __restrict__ part, R kick,
                                           long long step_off, V4<R>* pos_out, V4<R>* vel_out,
                                           int stats, VrBuf vr, AlchK<R> ak)
{
    __shared__ V4<R> tf[MAXCLS * MAXCLS];
    __shared__ V4<R> te[EN ? MAXCLS * MAXCLS : 1];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int gid = blk * WG + threadIdx.x;
    const int i = gid / LPB, s = gid % LPB;
    const bool valid = i < d.N;
    const int ii = valid ? i : 0;
    // entry k = m LPB + s of bead i sits at lane_base + 64 m (tiled list)
    constexpr int BG = 64 / LPB;
    const size_t lane_base = (size_t)(ii / BG) * ((size_t)d.Kcap * BG) + (size_t)(ii % BG) * LPB + s;
    const int* __restrict__ nb = (LIST == 1 ? d.nbr_in : d.nbr) + lane_base;
    int* __restrict__ nb_out = d.nbr_in + lane_base;
    const V4<R>* __restrict__ P = d.posq;
    constexpr int B = 4;
    constexpr int BT = B >= 8 ? 4 : 2;
    const int mcap = d.Kcap / LPB;
    // The bead, its count and its first batch of list entries (clamped to
    // the bead's tile) go out first, in one round trip with the parameter
    // table below.  Reads needed only after the walk (bonded records and
    // partners, the integrator's inputs) are issued after it: held across
    // the walk they would cost occupancy.
    const V4<R> pi = d.posq[ii];
    int jj0[B];
#pragma unroll
    for (int b = 0; b < B; ++b) jj0[b] = nb[(size_t)min(b, mcap - 1) * 64];
    int m1n;   // entries this lane walks
    if (LIST == 1) {
        m1n = valid ? min(d.ncnt_in[(size_t)i * LPB + s], mcap) : 0;
    } else {
        const int n1 = valid ? d.ncnt[i] : 0;
        m1n = n1 > s ? (n1 - s + LPB - 1) / LPB : 0;
    }
    // FUSE 1, 2, 3: after the forces, thread t < WG / LPB of the block integrates the
    // block's bead t (forces handed over through LDS), so that the
    // integrator runs on full waves instead of one lane per bead
    constexpr int NBB = WG / LPB;
    const int ib = blk * NBB + threadIdx.x;
    const bool integ = FUSE != 0 && threadIdx.x < NBB && ib < d.N;
    for (int t = threadIdx.x; t < MAXCLS * MAXCLS; t += WG) {
        tf[t] = d.tabF[t];
        if (EN) te[t] = d.tabE[t];
    }
    __syncthreads();
    const int ci = valid ? cls_of<R>(pi.w) : 0;
    const V4<R>* rowF = tf + ci * MAXCLS;
    const V4<R>* rowE = EN ? te + ci * MAXCLS : tf;
    R fx = 0, fy = 0, fz = 0;
    double elj = 0.0, erf = 0.0, eb = 0.0, ea = 0.0, ek = 0.0;
    double wp[3] = { 0.0, 0.0, 0.0 }, wb[3] = { 0.0, 0.0, 0.0 }, mv2[3] = { 0.0, 0.0, 0.0 };
    int np = 0;
    // list walk in batches of B entries per lane, then short batches of BT
    // for the tail, the batch sizes uniform over the wave; branch-free inside a
    // batch: all list reads, then all coordinate gathers (the bead itself for
    // unused slots), then the pair terms with their LDS parameter reads in
    // flight together
    int nkeep = 0;   // LIST 2: entries kept for the inner list
    int mmax = m1n;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mmax = max(mmax, __shfl_xor(mmax, o, 64));
    // one batch of pairs; SH: some entry of the wave carries a periodic
    // code, so bead i is shifted down by L along the code's axes (exact:
    // it sits in the upper half of the box there); the common case takes
    // bead i as it is
    auto pairs = [&](int m0, const int* jj, const V4<R>* q, auto nbt, auto shx) {
        constexpr int NB = decltype(nbt)::value;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bool live = m0 + b < m1n;
            R xs = pi.x, ys = pi.y, zs = pi.z;
            if (decltype(shx)::value) {
                const int code = live ? (int)((unsigned)jj[b] >> CODE_SHIFT) : 0;
                if (code & 1) xs -= d.L[0];
                if (code & 2) ys -= d.L[1];
                if (code & 4) zs -= d.L[2];
            }
            const R dx = xs - q[b].x, dy = ys - q[b].y, dz = zs - q[b].z;
            const R r2 = dx * dx + dy * dy + dz * dz;
            if (LIST == 2 && live && r2 < d.rin2) nb_out[(size_t)(nkeep++) * 64] = jj[b];
            // unused slots hold the bead itself (r2 = 0): rsq gives inf and
            // the terms inf or NaN, which the selects below drop
            const bool in = live && r2 < d.rc2;
            const R rinv = rsq<R>(r2);
            const R rinv2 = rinv * rinv;
            const R rinv6 = rinv2 * rinv2 * rinv2;
            const V4<R> p = rowF[cls_of<R>(q[b].w)];
            R fs = (p.y * rinv6 - p.x) * (rinv6 * rinv2) + (p.z * (rinv * rinv2) - p.w);
            fs = in ? fs : (R)0;
            fx += fs * dx;
            fy += fs * dy;
            fz += fs * dz;
            if (EN) {
                const V4<R> e = rowE[cls_of<R>(q[b].w)];
                const R vlj = (e.y * rinv6 - e.x) * rinv6 - e.w;
                const R vrf = e.z * (rinv + d.krf * r2 - d.crf);
                if (in) {
                    elj += (double)vlj;
                    erf += (double)vrf;
                    np += 1;
                    wp[0] += (double)(fs * dx) * (double)dx;
                    wp[1] += (double)(fs * dy) * (double)dy;
                    wp[2] += (double)(fs * dz) * (double)dz;
                }
            }
        }
    };
    // coordinates by 32-bit byte offset (slots < 2^27, checked at creation):
    // the shift code's bits fall off the top of the shifted entry
    constexpr int PSH = sizeof(V4<R>) == 16 ? 4 : 5;
    const char* __restrict__ Pc = reinterpret_cast<const char*>(P);
    auto compute = [&](int m0, const int* jj, auto nbt) {
        constexpr int NB = decltype(nbt)::value;
        V4<R> q[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const unsigned o = (unsigned)(m0 + b < m1n ? jj[b] : ii) << PSH;
            q[b] = *reinterpret_cast<const V4<R>*>(Pc + o);
        }
        bool shifted = false;
#pragma unroll
        for (int b = 0; b < NB; ++b) shifted |= (m0 + b < m1n) && (unsigned)jj[b] > (unsigned)JMASK;
        if (__ballot(shifted) != 0ull) pairs(m0, jj, q, nbt, std::true_type{});
        else pairs(m0, jj, q, nbt, std::false_type{});
    };
    auto batch = [&](int m0, auto nbt) {
        constexpr int NB = decltype(nbt)::value;
        int jj[NB];
        if constexpr (NB == B) {
            // full batches end at mmax <= mcap: no clamp, one base address
            const int* __restrict__ nbm = nb + (size_t)m0 * 64;
#pragma unroll
            for (int b = 0; b < NB; ++b) jj[b] = nbm[b * 64];
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) jj[b] = nb[(size_t)min(m0 + b, mcap - 1) * 64];
        }
        compute(m0, jj, nbt);
    };
    int m0 = 0;
    if (mmax > 0) {
        compute(0, jj0, std::integral_constant<int, B>{});
        m0 = B;
    }

    for (; m0 + B <= mmax; m0 += B) batch(m0, std::integral_constant<int, B>{});
    for (; m0 < mmax; m0 += BT) batch(m0, std::integral_constant<int, BT>{});
    // the integrator's inputs, in flight with the bonded terms and the
    // force reduction (loaded here, not up front, to keep registers free
    // during the walk)
    BeadPre<R> pre{};
    V4<R> pb{}, vk{};
    int grp = 0;   // coupling group of bead ib (a chain of four loads, in flight early)
    if (FUSE == 2 && integ) {
        vk = d.vel[ib];   // the closing half-kick's velocity
        grp = vr_group(d, vr, ib);
    }
    int af = 0;
    V4<R> gd{};   // FUSE 3: the bead's F_B - F_A
    if ((FUSE == 1 || FUSE == 3) && integ) {
        pb = d.posq[ib];
        pre = bead_pre(d, ib, LIST == 1);
        if (LIST == 2) pre.xri = pb;   // this pass makes the bead's coordinates the reference
        if (FUSE == 3) {
            af = ak.aff_flag[ib];
            if (af) gd = d.dfrc[ib];
        }
    }
    // bonded records (lane s takes terms s, s + LPB, ... of its bead) and
    // their partners' coordinates
    constexpr int TPL = (MAXBT + LPB - 1) / LPB;
    int4 bt[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u)
        bt[u] = (s + u * LPB < MAXBT) ? d.bslot[(size_t)ii * MAXBT + s + u * LPB]
                                      : make_int4(-1, ii, ii, 0);
    V4<R> b1[TPL], b2[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u) { b1[u] = P[bt[u].y]; b2[u] = P[bt[u].z]; }
    // bonded terms of bead i
#pragma unroll
    for (int u = 0; u < TPL; ++u)
        if (valid && bt[u].x >= 0)
            bonded_term<R, EN>(d, pi, bt[u], b1[u], b2[u], fx, fy, fz, eb, ea, wb);
    if (EN && valid && s == 0) {
        V4<R> v = d.vel[i];
        mv2[0] = (double)v.x * v.x / (double)v.w;
        mv2[1] = (double)v.y * v.y / (double)v.w;
        mv2[2] = (double)v.z * v.z / (double)v.w;
        ek = 0.5 * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z) / (double)v.w;
    }
#pragma unroll
    for (int m = LPB / 2; m >= 1; m >>= 1) {
        fx += __shfl_xor(fx, m);
        fy += __shfl_xor(fy, m);
        fz += __shfl_xor(fz, m);
    }
    if (!EN) {
        const bool own = valid && s == 0;
        if constexpr (FUSE == 0) {
            if (own) d.frc[i] = V4<R>{ fx, fy, fz, (R)0 };
        } else if constexpr (FUSE == 2) {
            __shared__ V4<R> fk[NBB];
            __shared__ double sk[4][WG / 64];
            if (own) {
                const V4<R> f{ fx, fy, fz, (R)0 };
                d.frc[i] = f;
                fk[threadIdx.x / LPB] = f;
            }
            __syncthreads();
            // only the first NIW waves integrate (thread t < NBB takes bead t)
            constexpr int NIW = (NBB + 63) / 64;
            if (threadIdx.x < NIW * 64) {   // wave-uniform
                double q[4] = { 0.0, 0.0, 0.0, 0.0 };   // K of group 0, 1; beads of group 0, 1
                if (integ) {
                    V4<R> v = vk;
                    const V4<R> f = fk[threadIdx.x];
                    v.x += kick * v.w * f.x; v.y += kick * v.w * f.y; v.z += kick * v.w * f.z;
                    d.vel[ib] = v;
                    const double k2 =
                        0.5 * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z) / (double)v.w;
                    const bool g1 = grp != 0;
                    q[0] = g1 ? 0.0 : k2; q[1] = g1 ? k2 : 0.0;
                    q[2] = g1 ? 0.0 : 1.0; q[3] = g1 ? 1.0 : 0.0;
                }
                // butterfly sums: every lane holds the wave's totals
                double x[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) x[c] = wave_sum(q[c]);
                const int l = threadIdx.x & 63;
                if constexpr (NIW == 1) {
                    if (l < 4) part[4 * blk + l] = l == 0 ? x[0] : l == 1 ? x[1] : l == 2 ? x[2] : x[3];
                } else {
                    if (l == 0)
                        for (int c = 0; c < 4; ++c) sk[c][threadIdx.x >> 6] = x[c];
                }
            }
            if constexpr (NIW > 1) {
                __syncthreads();
                if (threadIdx.x < 4) {
                    double t = 0.0;
                    for (int w = 0; w < NIW; ++w) t += sk[threadIdx.x][w];
                    part[4 * blk + threadIdx.x] = t;
                }
            }
        } else {
            __shared__ V4<R> fsh[NBB];
            if (LIST == 2 && valid) {
                d.ncnt_in[(size_t)i * LPB + s] = nkeep;
                if (s == 0) d.xref_in[i] = pi;
            }
            if (own) {
                const V4<R> f{ fx, fy, fz, (R)0 };
                if (FUSE == 1) d.frc[i] = f;
                fsh[threadIdx.x / LPB] = f;
            }
            if (FUSE == 3 && blockIdx.x == 0 && threadIdx.x == 0) ak.md[0] += ak.dlw * ak.md[1];
            __syncthreads();
            float e2 = 0.f, e2_in = 0.f;
            if (integ) {
                V4<R> f = fsh[threadIdx.x];
                if (FUSE == 3) {
                    if (af) { f.x += ak.lam * gd.x; f.y += ak.lam * gd.y; f.z += ak.lam * gd.z; }
                    pre.v.x += kick * pre.v.w * f.x; pre.v.y += kick * pre.v.w * f.y;
                    pre.v.z += kick * pre.v.w * f.z;
                    if (af) { f.x += ak.dl * gd.x; f.y += ak.dl * gd.y; f.z += ak.dl * gd.z; }
                    d.frc[ib] = f;
                }
                e2 = baoab_bead(d, ib, pb, pre, f, kick, step_off, pos_out, vel_out, LIST != 0, e2_in);
            }
            if (stats & 1) disp_stats_lead<(NBB + 63) / 64>(d, e2, e2_in, integ);
            if (FUSE == 1 && (stats & 2) && threadIdx.x < (NBB + 63) / 64 * 64) {   // wave-uniform
                int cell = -1;
                if (integ) {
                    V4<R> p = pos_out[ib];   // this thread's own store above
                    cell = bin_cell(d, p);
                    pos_out[ib] = p;
                }
                bin_place(d, ib, cell);
            }
        }
    } else {
        __shared__ double sh[16][WG / 64];
        double v[16] = { elj, erf, (double)np, eb, ea, ek, valid ? (double)m1n : 0.0,
                         wp[0], wp[1], wp[2], wb[0], wb[1], wb[2], mv2[0], mv2[1], mv2[2] };
        const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            double x = wave_sum(v[q]);
            if (l == 0) sh[q][w] = x;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            double acc = 0.0;
            for (int ww = 0; ww < WG / 64; ++ww) acc += sh[threadIdx.x][ww];
            part[16 * blk + threadIdx.x] = acc;
        }
    }
}

// Fixed-order float64 sum of the block partials:
// out = {lj, rf, bond, angle, kinetic, n_pairs, list entries, virial W_aa (3),
// sum m v_a^2 (3)}
__global__ void k_energy_final(const double* __restrict__ p, int nb, double* __restrict__ out)
{
    __shared__ double sh[16][256];
    int t = threadIdx.x;
    double a[16];
    for (int q = 0; q < 16; ++q) a[q] = 0.0;
    for (int b = t; b < nb; b += 256)
        for (int q = 0; q < 16; ++q) a[q] += p[16 * b + q];
    for (int q = 0; q < 16; ++q) sh[q][t] = a[q];
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (t < off)
            for (int q = 0; q < 16; ++q) sh[q][t] += sh[q][t + off];
        __syncthreads();
    }
    if (t == 0) {
        // every unordered pair appears twice in the full lists
        out[0] = 0.5 * sh[0][0];
        out[1] = 0.5 * sh[1][0];
        out[2] = sh[3][0];
        out[3] = sh[4][0];
        out[4] = sh[5][0];
        out[5] = 0.5 * sh[2][0];
        out[6] = sh[6][0];   // entries walked: pair slots of one force pass
        for (int a = 0; a < 3; ++a) {
            out[7 + a] = 0.5 * sh[7 + a][0] + sh[10 + a][0];
            out[10 + a] = sh[13 + a][0];
        }
    }
}

// ----------------------------------------------------------------- launch
template <typename R, int LPB, bool EN, int FUSE, int LIST>
static void nb_launch(const Dev<R>& d, double* part, R kick, long long step_off, V4<R>* pos_out,
                      V4<R>* vel_out, int stats, hipStream_t st, VrBuf vr = VrBuf{},
                      AlchK<R> ak = AlchK<R>{})
{
    int nthr = d.N * LPB;
    hipLaunchKernelGGL((k_nb<R, LPB, EN, FUSE, LIST>), dim3((nthr + WG - 1) / WG), dim3(WG), 0, st, d,
                       part, kick, step_off, pos_out, vel_out, stats, vr, ak);
}

// forces (energy=false) or energies into part (energy=true), Verlet list;
// returns blocks
template <typename R>
int launch_nonbonded(const Dev<R>& d, int lpb, bool energy, double* part, hipStream_t st)
{
    switch (lpb * 2 + (energy ? 1 : 0)) {
    case 2: nb_launch<R, 1, false, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 3: nb_launch<R, 1, true, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 4: nb_launch<R, 2, false, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 5: nb_launch<R, 2, true, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 8: nb_launch<R, 4, false, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 9: nb_launch<R, 4, true, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 16: nb_launch<R, 8, false, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    case 17: nb_launch<R, 8, true, 0, 0>(d, part, 0, 0, nullptr, nullptr, 0, st); break;
    default: break;
    }
    return (d.N * lpb + WG - 1) / WG;
}

// forces followed by the next step's B-A-O-A for every bead (see k_nb);
// list: 0 Verlet list, 1 inner list, 2 Verlet list + prune into the inner
// list (lanes per bead 2, 4 or 8; 1 walks the Verlet list)
template <typename R>
void launch_nonbonded_fused(const Dev<R>& d, int lpb, int list, R kick, long long step_off,
                            V4<R>* pos_out, V4<R>* vel_out, int stats, hipStream_t st)
{
#define NBF(L, M) nb_launch<R, L, false, 1, M>(d, nullptr, kick, step_off, pos_out, vel_out, stats, st)
    switch (lpb * 4 + list) {
    case 4: case 5: case 6: NBF(1, 0); break;
    case 8: NBF(2, 0); break;
    case 9: NBF(2, 1); break;
    case 10: NBF(2, 2); break;
    case 16: NBF(4, 0); break;
    case 17: NBF(4, 1); break;
    case 18: NBF(4, 2); break;
    case 32: NBF(8, 0); break;
    case 33: NBF(8, 1); break;
    case 34: NBF(8, 2); break;
    default: break;
    }
#undef NBF
}

// forces followed by velocity rescaling's closing half-kick with the block
// sums of the kinetic energies (see k_nb, FUSE 2); returns the blocks, i.e.
// the partials written to vr.part
template <typename R>
int launch_nonbonded_kick(const Dev<R>& d, int lpb, const VrBuf& vr, R kick, hipStream_t st)
{
    switch (lpb) {
    case 1: nb_launch<R, 1, false, 2, 0>(d, vr.part, kick, 0, nullptr, nullptr, 0, st, vr); break;
    case 2: nb_launch<R, 2, false, 2, 0>(d, vr.part, kick, 0, nullptr, nullptr, 0, st, vr); break;
    case 4: nb_launch<R, 4, false, 2, 0>(d, vr.part, kick, 0, nullptr, nullptr, 0, st, vr); break;
    case 8: nb_launch<R, 8, false, 2, 0>(d, vr.part, kick, 0, nullptr, nullptr, 0, st, vr); break;
    default: return 0;
    }
    return (d.N * lpb + WG - 1) / WG;
}

// MDAS segment boundary fused into the force pass (see k_nb, FUSE 3):
// Verlet list, kick = dt / 2, the update written to pos_out
template <typename R>
void launch_nonbonded_alch(const Dev<R>& d, int lpb, R kick, long long step_off, V4<R>* pos_out,
                           V4<R>* vel_out, const AlchK<R>& ak, hipStream_t st)
{
#define NBA(L) nb_launch<R, L, false, 3, 0>(d, nullptr, kick, step_off, pos_out, vel_out, 1, st, VrBuf{}, ak)
    switch (lpb) {
    case 1: NBA(1); break;
    case 2: NBA(2); break;
    case 4: NBA(4); break;
    case 8: NBA(8); break;
    default: break;
    }
#undef NBA
}

void launch_energy_final(const double* p, int nb, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, st, p, nb, out);
}

template void launch_nonbonded_alch<float>(const Dev<float>&, int, float, long long, V4<float>*,
                                           V4<float>*, const AlchK<float>&, hipStream_t);
template void launch_nonbonded_alch<double>(const Dev<double>&, int, double, long long, V4<double>*,
                                            V4<double>*, const AlchK<double>&, hipStream_t);
template int launch_nonbonded<float>(const Dev<float>&, int, bool, double*, hipStream_t);
template int launch_nonbonded_kick<float>(const Dev<float>&, int, const VrBuf&, float, hipStream_t);
template int launch_nonbonded_kick<double>(const Dev<double>&, int, const VrBuf&, double, hipStream_t);
template int launch_nonbonded<double>(const Dev<double>&, int, bool, double*, hipStream_t);
template void launch_nonbonded_fused<float>(const Dev<float>&, int, int, float, long long,
                                            V4<float>*, V4<float>*, int, hipStream_t);
template void launch_nonbonded_fused<double>(const Dev<double>&, int, int, double, long long,
                                             V4<double>*, V4<double>*, int, hipStream_t);

}  // namespace mbx
