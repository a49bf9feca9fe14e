// Per-image cell lists and full neighbour lists.
//
// The neighbours of atom i are every (j, n) != (i, 0) with
//     r = (R_j - R_i) + ((n0 h_0 + n1 h_1) + n2 h_2),  (r_x r_x + r_y r_y) + r_z r_z < rc^2,
// evaluated in FP64 with every operation rounded on its own (no contraction), on the
// unwrapped positions R = R~ D.  Bins only generate candidates, so the set does not
// depend on the binning.  This is the local environment of Sec. II.B, Eq. (4).
//
// Kernels, in order, one grid row per image:
//   k_bin_assign  R = R~ D, wrapped fractional coordinate, bin id, integer counts
//   k_bin_scan    exclusive prefix sum of the counts (one block per image); zeroes counts
//   k_bin_fill    atoms into bins (atomic cursors)
//   k_bin_sort    sort each bin by atom index, so the lists are deterministic
//   k_nlist       stencil walk, exact inclusion test, packed entry-major lists
#include "cfneb_dev.h"

namespace cfneb {

__device__ inline size_t bin_base(const BandDev& b, int slot) { return size_t(slot) * (b.nbcap + 1); }

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_assign(BandDev b, int all_images)
{
    const BandState* st = b.st;
    const int k = blockIdx.y;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images) || i >= b.N) return;
    const int slot = st->slot[k];
    const ImageGeom& g = b.geom[slot];
    const double* X = Xs(b, slot);
    const double x = X[i], y = X[b.ld + i], z = X[2 * size_t(b.ld) + i];
    double r[3];
    for (int c = 0; c < 3; ++c) r[c] = (x * g.D[c] + y * g.D[3 + c]) + z * g.D[6 + c];
    double* R = Rs(b, slot);
    R[i] = r[0];
    R[b.ld + i] = r[1];
    R[2 * size_t(b.ld) + i] = r[2];
    int bi[3], img[3];
    for (int q = 0; q < 3; ++q) {
        const double s = (r[0] * g.hinv[q] + r[1] * g.hinv[3 + q]) + r[2] * g.hinv[6 + q];
        double fl = floor(s);
        if (!isfinite(fl) || fabs(fl) > 1e6) fl = 0.0;  // non-finite input: caught by the energy check
        img[q] = int(fl);
        const double sw = s - fl;
        int bq = int(floor(sw * g.nb[q]));
        bq = bq < 0 ? 0 : (bq >= g.nb[q] ? g.nb[q] - 1 : bq);
        bi[q] = bq;
    }
    const int bin = (bi[0] * g.nb[1] + bi[1]) * g.nb[2] + bi[2];
    b.binfo[size_t(slot) * b.N + i] = make_int4(bin, img[0], img[1], img[2]);
    atomicAdd(&b.bcount[bin_base(b, slot) + bin], 1);
}

// One block of 1024 threads per image: each thread owns a contiguous run of bins.
__global__ void __launch_bounds__(1024) k_bin_scan(BandDev b, int all_images)
{
    const BandState* st = b.st;
    const int k = blockIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int slot = st->slot[k];
    const int nbins = b.geom[slot].nbins;
    int* cnt = b.bcount + bin_base(b, slot);
    int* start = b.bstart + bin_base(b, slot);
    int* cur = b.bcursor + bin_base(b, slot);
    const int t = threadIdx.x;
    const int chunk = (nbins + 1023) / 1024;
    const int lo = min(t * chunk, nbins), hi = min(lo + chunk, nbins);
    int local = 0;
    for (int p = lo; p < hi; ++p) local += cnt[p];
    // block exclusive scan: wave inclusive scan, then the 16 wave totals
    __shared__ int wsum[16];
    const int lane = t & 63, wid = t >> 6;
    int incl = local;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wid; ++w) base += wsum[w];
    int run = base + incl - local;
    for (int p = lo; p < hi; ++p) {
        start[p] = run;
        cur[p] = run;
        run += cnt[p];
        cnt[p] = 0;
    }
    if (t == 1023) start[nbins] = base + incl;
}

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_fill(BandDev b, int all_images)
{
    BandState* st = b.st;
    const int k = blockIdx.y;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images) || i >= b.N) return;
    const int slot = st->slot[k];
    const int bin = b.binfo[size_t(slot) * b.N + i].x;
    const int pos = atomicAdd(&b.bcursor[bin_base(b, slot) + bin], 1);
    if (pos >= 0 && pos < b.N)
        b.batoms[size_t(slot) * b.N + pos] = i;
}

__global__ void __launch_bounds__(CFNEB_TILE) k_bin_sort(BandDev b, int all_images)
{
    const BandState* st = b.st;
    const int k = blockIdx.y;
    const int bin = blockIdx.x * CFNEB_TILE + threadIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images)) return;
    const int slot = st->slot[k];
    if (bin >= b.geom[slot].nbins) return;
    const int* start = b.bstart + bin_base(b, slot);
    int* a = b.batoms + size_t(slot) * b.N;
    const int lo = start[bin], hi = min(start[bin + 1], b.N);
    for (int p = lo + 1; p < hi; ++p) {
        const int v = a[p];
        int q = p - 1;
        while (q >= lo && a[q] > v) {
            a[q + 1] = a[q];
            --q;
        }
        a[q + 1] = v;
    }
}

__device__ inline int floordiv_i(int a, int m) { return (a >= 0) ? a / m : -((-a + m - 1) / m); }

// Exact squared distance of entry (j, n); every operation rounded separately.
__device__ inline double exact_r2(const double* ri, const double* rj, const double* h, int n0,
                                  int n1, int n2, double* d)
{
#pragma clang fp contract(off)
    for (int c = 0; c < 3; ++c) {
        const double sh = (double(n0) * h[c] + double(n1) * h[3 + c]) + double(n2) * h[6 + c];
        d[c] = (rj[c] - ri[c]) + sh;
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

template <typename T, bool STORE_BONDS>
__global__ void __launch_bounds__(CFNEB_TILE) k_nlist(BandDev b, int all_images)
{
    BandState* st = b.st;
    const int k = blockIdx.y;
    const int i = blockIdx.x * CFNEB_TILE + threadIdx.x;
    if (band_stopped(st) || !image_active(st, k, all_images) || i >= b.N) return;
    const int slot = st->slot[k];
    const ImageGeom& g = b.geom[slot];
    const double* R = Rs(b, slot);
    const int4* info = b.binfo + size_t(slot) * b.N;
    const int* start = b.bstart + bin_base(b, slot);
    const int* atoms = b.batoms + size_t(slot) * b.N;
    const size_t N = b.N;
    uint32_t* nbr = b.nbr + size_t(slot) * b.cap * N;
    using T4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
    T4* dvec = STORE_BONDS ? reinterpret_cast<T4*>(b.dvec) + size_t(slot) * b.cap * N : nullptr;

    double h[9];
    for (int q = 0; q < 9; ++q) h[q] = g.h[q];
    const double ri[3] = {R[i], R[b.ld + i], R[2 * size_t(b.ld) + i]};
    const int4 me = info[i];
    const int nb0 = g.nb[0], nb1 = g.nb[1], nb2 = g.nb[2];
    const int b0 = me.x / (nb1 * nb2), b1 = (me.x / nb2) % nb1, b2 = me.x % nb2;
    int cnt = 0;
    bool bad_shift = false;
    for (int dx = -g.reach[0]; dx <= g.reach[0]; ++dx) {
        const int v0 = b0 + dx, m0 = floordiv_i(v0, nb0), a0 = v0 - m0 * nb0;
        for (int dy = -g.reach[1]; dy <= g.reach[1]; ++dy) {
            const int v1 = b1 + dy, m1 = floordiv_i(v1, nb1), a1 = v1 - m1 * nb1;
            for (int dz = -g.reach[2]; dz <= g.reach[2]; ++dz) {
                const int v2 = b2 + dz, m2 = floordiv_i(v2, nb2), a2 = v2 - m2 * nb2;
                const int bin = (a0 * nb1 + a1) * nb2 + a2;
                const int lo = start[bin], hi = min(start[bin + 1], b.N);
                for (int p = lo; p < hi; ++p) {
                    const int j = atoms[p];
                    const int4 oj = info[j];
                    const int n0 = m0 + me.y - oj.y;
                    const int n1 = m1 + me.z - oj.z;
                    const int n2 = m2 + me.w - oj.w;
                    if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                    const double rj[3] = {R[j], R[b.ld + j], R[2 * size_t(b.ld) + j]};
                    double d[3];
                    const double r2 = exact_r2(ri, rj, h, n0, n1, n2, d);
                    if (!(r2 < b.rc2)) continue;
                    if (abs(n0) > CFNEB_MAX_SHIFT || abs(n1) > CFNEB_MAX_SHIFT || abs(n2) > CFNEB_MAX_SHIFT) {
                        bad_shift = true;
                        continue;
                    }
                    if (cnt < b.cap) {
                        nbr[size_t(cnt) * N + i] = pack_nbr(j, n0, n1, n2);
                        if (STORE_BONDS) {
                            T4 e;
                            e.x = T(d[0]);
                            e.y = T(d[1]);
                            e.z = T(d[2]);
                            e.w = T(sqrt(r2));
                            dvec[size_t(cnt) * N + i] = e;
                        }
                    }
                    ++cnt;
                }
            }
        }
    }
    b.ncnt[size_t(slot) * N + i] = cnt;
    if (bad_shift) set_error(st, CFNEB_ECELL);
    if (cnt > b.cap) set_error(st, CFNEB_ENEIGH);
}

void launch_bins(const BandDev& b, int all_images, hipStream_t s)
{
    const dim3 gA(b.ntA, b.Mcap);
    k_bin_assign<<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    k_bin_scan<<<b.Mcap, 1024, 0, s>>>(b, all_images);
    k_bin_fill<<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    const dim3 gB((b.nbcap + CFNEB_TILE - 1) / CFNEB_TILE, b.Mcap);
    k_bin_sort<<<gB, CFNEB_TILE, 0, s>>>(b, all_images);
}

void launch_list(const BandDev& b, int all_images, hipStream_t s)
{
    const dim3 gA(b.ntA, b.Mcap);
    if (b.potential == CFNEB_TERSOFF_C) {
        if (b.fp64)
            k_nlist<double, true><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
        else
            k_nlist<float, true><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    } else {
        k_nlist<double, false><<<gA, CFNEB_TILE, 0, s>>>(b, all_images);
    }
}

void launch_nlist(const BandDev& b, int all_images, hipStream_t s)
{
    launch_bins(b, all_images, s);
    launch_list(b, all_images, s);
}

}  // namespace cfneb
