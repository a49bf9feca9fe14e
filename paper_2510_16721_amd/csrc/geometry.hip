// Cell-filter geometry of every image and band construction (Sec. II.C).
//
// Per image: B = (cell rows of X) / c_f, D = symsqrt(B) (the rotation-free gauge,
// Eq. (15)), h = h0 D, h^-1, Omega = |det h|, the perpendicular widths of the cell
// and the bin grid of the cell list.
#include "cfneb_dev.h"

namespace cfneb {

// Symmetric positive square root by cyclic Jacobi rotations on the symmetric part.
// Returns false if an eigenvalue is not positive.
__device__ __forceinline__ bool sym_sqrt(const double* Bin, double* D)
{
    double a[3][3], q[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = 0.5 * (Bin[3 * i + j] + Bin[3 * j + i]);
            q[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int it = 0; it < 64; ++it) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double on = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-36 * on) break;
#pragma unroll
        for (int pr = 0; pr < 3; ++pr) {
            const int p = (pr == 2) ? 1 : 0;
            const int r = (pr == 0) ? 1 : 2;
            const double apr = a[p][r];
            if (apr == 0.0) continue;
            const double th = (a[r][r] - a[p][p]) / (2.0 * apr);
            const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = rsqrt(t * t + 1.0);
            const double s = t * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = a[k][p], y = a[k][r];
                a[k][p] = c * x - s * y;
                a[k][r] = s * x + c * y;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = a[p][k], y = a[r][k];
                a[p][k] = c * x - s * y;
                a[r][k] = s * x + c * y;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double x = q[k][p], y = q[k][r];
                q[k][p] = c * x - s * y;
                q[k][r] = s * x + c * y;
            }
        }
    }
    double rt[3];
    for (int i = 0; i < 3; ++i) {
        if (!(a[i][i] > 0.0)) return false;
        rt[i] = sqrt(a[i][i]);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            D[3 * i + j] = q[i][0] * rt[0] * q[j][0] + q[i][1] * rt[1] * q[j][1] + q[i][2] * rt[2] * q[j][2];
    return true;
}

__device__ __forceinline__ bool image_geometry(const BandDev& b, const double* X, ImageGeom& g)
{
    double B[9];
    const double icf = 1.0 / b.cf;
    for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) B[3 * q + c] = X[size_t(c) * b.ld + b.N + q] * icf;
    if (b.cell_filter == 1) {
        // D-variant: the cell rows hold c_f D itself (rotations included)
        for (int q = 0; q < 9; ++q) g.D[q] = B[q];
        const double det = det3(g.D);
        if (!(det > 0.0) || !isfinite(det)) return false;
    } else if (!sym_sqrt(B, g.D)) {
        return false;
    }
    inv3(g.D, g.Dinv);
    mm3(b.h0, g.D, g.h);
    inv3(g.h, g.hinv);
    g.omega = fabs(det3(g.h));
    if (!(g.omega > 0.0) || !isfinite(g.omega)) return false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double* u = g.h + 3 * ((k + 1) % 3);
        const double* v = g.h + 3 * ((k + 2) % 3);
        const double cx = u[1] * v[2] - u[2] * v[1];
        const double cy = u[2] * v[0] - u[0] * v[2];
        const double cz = u[0] * v[1] - u[1] * v[0];
        g.w[k] = g.omega / sqrt(cx * cx + cy * cy + cz * cz);
    }
    // Bins along fractional axis k have perpendicular width w_k / nb_k >= rcl / sub
    // (1 + 1e-9), rcl = rc + skin the candidate cutoff, so a +-sub bin stencil holds
    // every pair closer than rcl.  Dense systems (at least 8 atoms per rcl^3, e.g. LJ
    // near its minimum: about 24) take sub = 2: the 5^3 stencil of half-width bins
    // tests about 0.58 of the pairs the 3^3 stencil does, and candidates come in finer
    // spatial order; sparse ones (carbon: about 3) keep sub = 1, where half-width bins
    // would be mostly empty.  Cells narrower than that get one bin and a stencil wide
    // enough for all the periodic images needed.
    const int sub = (double(b.N) * b.rcl * b.rcl * b.rcl >= 8.0 * g.omega) ? 2 : 1;
    g.sub = sub;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double q = g.w[k] * sub / (b.rcl * (1.0 + 1e-9));
        if (q >= double(sub)) {
            g.nb[k] = int(fmin(floor(q), 1024.0));
            g.reach[k] = sub;
        } else {
            g.nb[k] = 1;
            g.reach[k] = int(ceil(b.rcl / g.w[k])) + 1;
        }
    }
    // (scalar counts: an array indexed at run time would keep the whole geometry
    // record in scratch memory)
    int n0 = g.nb[0], n1 = g.nb[1], n2 = g.nb[2];
    while (n0 * n1 * n2 > b.nbcap) {
        // the first of the largest counts loses a bin; wider bins keep the +-1
        // stencil valid
        if (n1 > n0 && n1 >= n2)
            --n1;
        else if (n2 > n0 && n2 > n1)
            --n2;
        else
            --n0;
    }
    g.nb[0] = n0;
    g.nb[1] = n1;
    g.nb[2] = n2;
    g.nbins = n0 * n1 * n2;
    for (int k = 0; k < 3; ++k)
        if (g.reach[k] > 8) return false;  // shifts beyond the 4-bit packing
    return true;
}

// Between candidate builds every candidate is closer than rcl + skin (the skin test
// rebuilds before 2 max|displacement| + rcl |E| reaches the skin), so when that stays
// under half of each perpendicular width w_k, every candidate's fractional separation
// is inside (-1/2, 1/2) and the wrapped 32-bit fixed-point difference is exact.
// The separation from such a difference (3x3 product with h 2^-32 in FP64, within
// 3 2^-53 kappa |d|, kappa = |h|_F |h^-1|_F; 2^-32 sqrt(3) |h|_F from rounding the
// coordinates), rounded to FP32 and squared in FP32 (u = 2^-24: within 8u relative
// in r^2), gives an r^2 within twice that relative bound (taken at |d| = rc) of the
// exact one; the band around rc^2 where the FP64 test decides is twice that again.
__device__ __forceinline__ void fixed_point_bounds(const BandDev& b, ImageGeom& g)
{
    double hf = 0.0, hif = 0.0;
    for (int q = 0; q < 9; ++q) {
        hf += g.h[q] * g.h[q];
        hif += g.hinv[q] * g.hinv[q];
    }
    hf = sqrt(hf);
    hif = sqrt(hif);
    const double u = 0x1p-24;
    const double rel = 2.0 * (8.0 * u + 2.0 * (3.0 * 0x1p-53 * hf * hif + 0x1p-32 * 1.7320508075688772 * hf / b.rc));
    const double wmin = fmin(g.w[0], fmin(g.w[1], g.w[2]));
    g.wrap = (g.err == 0 && rel < 1e-3 && (b.rcl + b.skin) * (1.0 + 1e-6) < 0.5 * wmin) ? 1 : 0;
    g.r2lo = float(b.rc2 * (1.0 - rel));
    g.r2hi = float(b.rc2 * (1.0 + rel));
}

// Geometry of image k of band b and its strain since the candidate build; in a step,
// first the pending move of the image's cell rows.
__device__ __forceinline__ void geom_image(const BandDev& b, BandState* st, int k, int all_images)
{
    // the band state's fields read here are not written by this kernel
    const cmem<BandState>* sr = cp(st);
    const int slot = sr->slot[k];
    if (move_pending(sr, all_images)) {
        gmem<double>* X = gp(Xs(b, slot));
        const gmem<const double>* V = gp<const double>(Vs(b, sr->vcur, slot));
        const double sc = sr->scale, dt = sr->dt;
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) {
                const size_t o = size_t(c) * b.ld + b.N + q;
                X[o] += sc * (dt * V[o]);
            }
    }
    ImageGeom g;
    g.err = 0;
    if (!image_geometry(b, Xs(b, slot), g)) {
        g.err = 1;
        set_error(st, CFNEB_ECELL);
    }
    // strain since the candidate build: E = h_ref^-1 h - I
    const cmem<SkinState>& sk = *cp(b.skst + slot);
    g.enorm = 0.0;
    if (sk.valid) {
        double hri[9];
        for (int q = 0; q < 9; ++q) hri[q] = sk.hrefinv[q];
        mm3(hri, g.h, g.E);
        for (int q = 0; q < 3; ++q) g.E[4 * q] -= 1.0;
        for (int q = 0; q < 9; ++q) g.enorm += g.E[q] * g.E[q];
        g.enorm = sqrt(g.enorm);
    } else {
        for (int q = 0; q < 9; ++q) g.E[q] = 0.0;
    }
    fixed_point_bounds(b, g);
    b.geom[slot] = g;
}

// One block per band, one thread per image; the bands are taken from the table
// directly, so block 0 can write the step's work plan (every later kernel of the
// step walks it) in the same launch, alongside the geometry of the other blocks.
__global__ void __launch_bounds__(CFNEB_MAX_BANDS) k_geom(BatchDev bd, int all_images)
{
    // block 0 writes the plan while the others take the bands (grids of at least 8)
    if (blockIdx.x == 0) {
        plan_block(bd, all_images, 0);
        return;
    }
    for (int t = int(blockIdx.x) - 1; t < bd.cap; t += int(gridDim.x) - 1) {
        if (!bd.live[t]) continue;
        const BandDev& b = bd.bands[t];
        BandState* st = b.st;
        const int k = threadIdx.x;
        if (band_stopped(st) || k >= b.Mcap || !image_active(st, k, all_images)) continue;
        geom_image(b, st, k, all_images);
    }
}

// ---------------------------------------------------------------- construction
// staging: RA (3N, row-major) | RB (3N) | hA (9) | hB (9) | BB (9) | h0inv (9) | hBinv (9)
//          | D_B (9)
__global__ void k_init_endpoints(BandDev b)
{
    double* sg = b.staging + 6 * size_t(b.N);
    const double* hB = sg + 9;
    double* BB = sg + 18;
    double* h0inv = sg + 27;
    double* hBinv = sg + 36;
    double* Dr = sg + 45;
    inv3(b.h0, h0inv);
    inv3(hB, hBinv);
    double DrT[9];
    mm3(h0inv, hB, Dr);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) DrT[3 * i + j] = Dr[3 * j + i];
    mm3(Dr, DrT, BB);
}

__global__ void k_init_images(BandDev b, int M)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (r >= b.N + 3 || k >= M) return;
    const double* RA = b.staging;
    const double* RB = b.staging + 3 * size_t(b.N);
    const double* sg = b.staging + 6 * size_t(b.N);
    const double* BB = sg + 18;
    const double* h0inv = sg + 27;
    const double* hBinv = sg + 36;
    const double* Dr = sg + 45;
    double xa[3], xb[3];
    if (r < b.N) {
        const double* a = RA + 3 * size_t(r);
        const double* c = RB + 3 * size_t(r);
        double ds[3];
        for (int q = 0; q < 3; ++q) {
            const double sa = a[0] * h0inv[q] + a[1] * h0inv[3 + q] + a[2] * h0inv[6 + q];
            const double sb = c[0] * hBinv[q] + c[1] * hBinv[3 + q] + c[2] * hBinv[6 + q];
            ds[q] = sb - sa;
            ds[q] -= rint(ds[q]);
        }
        for (int q = 0; q < 3; ++q) {
            xa[q] = a[q];
            xb[q] = a[q] + (ds[0] * b.h0[q] + ds[1] * b.h0[3 + q] + ds[2] * b.h0[6 + q]);
        }
    } else {
        const int row = r - b.N;
        for (int q = 0; q < 3; ++q) {
            xa[q] = (row == q) ? b.cf : 0.0;
            // rotation-free filter: B of the final cell; D-variant: its D = h0^-1 h_B
            xb[q] = b.cf * (b.cell_filter == 1 ? Dr[3 * row + q] : BB[3 * row + q]);
        }
    }
    double* X = Xs(b, k);
    const double t = double(k) / double(M - 1);
    {
#pragma clang fp contract(off)
        for (int q = 0; q < 3; ++q) {
            double x;
            if (k == 0)
                x = xa[q];
            else if (k == M - 1)
                x = xb[q];
            else
                x = xa[q] + t * (xb[q] - xa[q]);
            X[size_t(q) * b.ld + r] = x;
        }
    }
}

__global__ void k_init_state(BandDev b, int M)
{
    BandState* st = b.st;
    st->M = M;
    for (int k = 0; k < CFNEB_MAX_IMAGES; ++k) st->slot[k] = (k < b.Mcap) ? k : 0;
    st->vcur = 0;
    st->step = 0;
    st->steps_call = 0;
    st->done = 0;
    st->err = 0;
    st->ci = -1;
    st->fresh = 1;
    st->n_pos = 0;
    st->alpha = b.astart;
    st->dt = b.dt0;
    st->f_tol = 0.0;
    st->fmax = 0.0;
    st->move = 0;
    st->refine_due = 0;
    st->ins = st->del = -1;
    st->changed = 0;
}

// Positions and cell of one logical image from the current coordinates.
__global__ void k_image_geom_one(BandDev b, int k)
{
    BandState* st = b.st;
    if (k < 0 || k >= st->M) return;
    ImageGeom g;
    const bool ok = image_geometry(b, Xs(b, st->slot[k]), g);
    double* out = b.staging + 3 * size_t(b.N);
    for (int q = 0; q < 9; ++q) out[q] = ok ? g.h[q] : 0.0;
    for (int q = 0; q < 9; ++q) out[9 + q] = ok ? g.D[q] : 0.0;
}

__global__ void k_image_positions(BandDev b, int k)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    BandState* st = b.st;
    if (i >= b.N || k < 0 || k >= st->M) return;
    const double* X = Xs(b, st->slot[k]);
    const double* D = b.staging + 3 * size_t(b.N) + 9;
    const double x = X[i], y = X[b.ld + i], z = X[2 * size_t(b.ld) + i];
    for (int c = 0; c < 3; ++c) b.staging[3 * size_t(i) + c] = x * D[c] + y * D[3 + c] + z * D[6 + c];
}

void launch_init_endpoints(const BandDev& b, hipStream_t s) { k_init_endpoints<<<1, 1, 0, s>>>(b); }

void launch_init_images(const BandDev& b, int M, hipStream_t s)
{
    dim3 grid((b.N + 3 + CFNEB_TILE - 1) / CFNEB_TILE, M);
    k_init_images<<<grid, CFNEB_TILE, 0, s>>>(b, M);
}

void launch_init_state(const BandDev& b, int M, hipStream_t s) { k_init_state<<<1, 1, 0, s>>>(b, M); }

// Geometry of the active images and the step's work plan (no separate plan launch).
void launch_geom(const Launch& L, int all_images, hipStream_t s)
{
    k_geom<<<L.g[KIND_BAND], CFNEB_MAX_BANDS, 0, s>>>(L.bd, all_images);
}

void launch_image_positions(const BandDev& b, int k, hipStream_t s)
{
    k_image_geom_one<<<1, 1, 0, s>>>(b, k);
    k_image_positions<<<(b.N + CFNEB_TILE - 1) / CFNEB_TILE, CFNEB_TILE, 0, s>>>(b, k);
}

}  // namespace cfneb
