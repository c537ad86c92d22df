// k_obs.hip -- the mixing observable: lateral pair histogram of the PO4
// beads of one lipid kind within each leaflet (Results: the pair
// correlation of like lipids' phosphates, whose highest peak follows the
// mixing).  Integer counts; the bin of a pair is decided on its float64
// squared lateral distance against a table of squared bin edges, so the
// result does not depend on the order of the pairs or on rounding inside a
// square root.
#include "membx_dev.h"

namespace mbx {

constexpr int OBS_TB = 256;     // points per tile of the pair kernel

// The selected molecules' PO4 coordinates (x, y in float64) and leaflets,
// compacted in arbitrary order (the histogram does not depend on it).
template <typename R>
__global__ void k_obs_gather(Dev<R> d, ObsBuf o, int kind, int po4)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.nm) return;
    const int lf = o.leaf[m];
    if (d.mol_kind[m] != kind || lf < 0) return;
    const V4<R> p = d.posq[d.inv[d.mol_first[m] + po4]];
    const int k = atomicAdd(o.n, 1);
    o.xy[k] = make_double2((double)p.x, (double)p.y);
    o.lf[k] = lf;
}

// Tile (ti, tj), ti <= tj, of all unordered pairs: thread t takes point
// ti * TB + t against the points of tile tj (staged in LDS), counts into an
// LDS histogram, then the work-group adds its non-empty bins to the global
// ones (64-bit integer atomics: exact in any order).
__global__ __launch_bounds__(OBS_TB) void k_obs_pairs(ObsBuf o, int npts, int nb, double w, double Lx,
                                                      double Ly)
{
    extern __shared__ __align__(8) unsigned char obs_lds[];
    double* e2 = reinterpret_cast<double*>(obs_lds);                  // [nb + 1]
    unsigned* hist = reinterpret_cast<unsigned*>(e2 + nb + 1);        // [nb]
    __shared__ double2 pj[OBS_TB];
    __shared__ int lj[OBS_TB];
    const int ti = blockIdx.x, tj = blockIdx.y, t = threadIdx.x;
    if (ti > tj) return;
    for (int k = t; k <= nb; k += OBS_TB) e2[k] = o.edge2[k];
    for (int k = t; k < nb; k += OBS_TB) hist[k] = 0u;
    const int j0 = tj * OBS_TB, i = ti * OBS_TB + t;
    if (j0 + t < npts) { pj[t] = o.xy[j0 + t]; lj[t] = o.lf[j0 + t]; }
    __syncthreads();
    if (i < npts) {
        const double2 pi = o.xy[i];
        const int li = o.lf[i];
        const int jn = min(OBS_TB, npts - j0);
        for (int jj = 0; jj < jn; ++jj) {
            if (j0 + jj <= i || lj[jj] != li) continue;
            double d2;
            {
#pragma clang fp contract(off)
                double dx = pi.x - pj[jj].x, dy = pi.y - pj[jj].y;
                if (dx > 0.5 * Lx) dx -= Lx;
                else if (dx < -0.5 * Lx) dx += Lx;
                if (dy > 0.5 * Ly) dy -= Ly;
                else if (dy < -0.5 * Ly) dy += Ly;
                d2 = dx * dx + dy * dy;
            }
            int k = (int)fmin(sqrt(d2) / w, (double)nb);
            while (k > 0 && e2[k] > d2) --k;
            while (k < nb && e2[k + 1] <= d2) ++k;
            if (k < nb) atomicAdd(&hist[k], 1u);
        }
    }
    __syncthreads();
    for (int k = t; k < nb; k += OBS_TB)
        if (hist[k]) atomicAdd(o.hist + k, (unsigned long long)hist[k]);
}

template <typename R>
void launch_obs_gather(const Dev<R>& d, const ObsBuf& o, int kind, int po4, hipStream_t st)
{
    hipLaunchKernelGGL(k_obs_gather<R>, dim3((d.nm + 255) / 256), dim3(256), 0, st, d, o, kind, po4);
}

void launch_obs_pairs(const ObsBuf& o, int npts, int nb, double w, double Lx, double Ly, hipStream_t st)
{
    const int T = (npts + OBS_TB - 1) / OBS_TB;
    if (T == 0) return;
    const size_t lds = sizeof(double) * (nb + 1) + sizeof(unsigned) * nb;
    hipLaunchKernelGGL(k_obs_pairs, dim3(T, T), dim3(OBS_TB), lds, st, o, npts, nb, w, Lx, Ly);
}

template void launch_obs_gather<float>(const Dev<float>&, const ObsBuf&, int, int, hipStream_t);
template void launch_obs_gather<double>(const Dev<double>&, const ObsBuf&, int, int, hipStream_t);

}  // namespace mbx
