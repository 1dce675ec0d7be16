// gfx950 kernels of libbd3mg: the per-block work of one BD3MG update
// (Sec. 2.3, box "Worker", for the criterion of Sec. 3.1).
//
// Layout: volumes are [nz][ny][nx], x fastest.  A workgroup owns a TX x TY
// tile of every slice it touches and marches along z through its segment:
// each global row it reads is 64 consecutive elements (one wavefront, fully
// coalesced), in-slice halos are staged through LDS, and the separable
// depth-variant blur is applied as an x pass then a y pass in LDS.  The
// z-direction of H^T is carried in a register ring of KZ partial sums.
//
// Inner products are accumulated in double: per thread in index order, then a
// wavefront shuffle tree, then the four wavefronts in order, then the
// workgroup slots of a block in slot order (k_solve) -- a fixed order, so
// every run gives bitwise identical results.
#include "bd3mg_internal.h"

namespace bd3mg {

namespace {

constexpr int LW = TX + 2 * RMAX;  // LDS row stride of halo tiles
constexpr int LH = TY + 2 * RMAX;  // LDS rows of halo tiles
constexpr int XW = TX + 2;         // iterate tile with a 1-voxel halo
constexpr int XH = TY + 2;
constexpr int ROWS_PER_THREAD = TY / (NT / TX);  // 4

__device__ __forceinline__ size_t vidx(const Geom &g, int k, int j, int i)
{
    return ((size_t)k * g.ny + j) * g.nx + i;
}

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Fill a (TY+2R) x (TX+2R) halo tile with f(j, i) at global (j, i) =
// (y0 - R + jj, x0 - R + ii); zero outside the slice.
template <typename T, typename F>
__device__ __forceinline__ void fill_halo(T *A, int x0, int y0, int R, const Geom &g, F f)
{
    const int w = TX + 2 * R, tot = w * (TY + 2 * R);
    for (int e = threadIdx.x; e < tot; e += NT) {
        const int jj = e / w, ii = e - jj * w;
        const int j = y0 - R + jj, i = x0 - R + ii;
        A[jj * LW + ii] = (i >= 0 && i < g.nx && j >= 0 && j < g.ny) ? f(j, i) : T(0);
    }
}

// x pass of the in-slice blur over rows [R - ry, R + TY + ry) of A into B.
// Forward (H):   B[jb][i] = sum_a wx[a + rx] A[.][i + R - a]
// Adjoint (H^T): B[jb][i] = sum_a wx[a + rx] A[.][i + R + a]
template <typename T, bool ADJ>
__device__ __forceinline__ void xpass(const T *A, T *B, const T *__restrict__ wx, int rx, int ry,
                                      int R)
{
    const int i = threadIdx.x & (TX - 1);
    const int rows = TY + 2 * ry;
    for (int jb = threadIdx.x / TX; jb < rows; jb += NT / TX) {
        const T *row = A + (jb + R - ry) * LW + i + R;
        T acc = 0;
        for (int a = -rx; a <= rx; ++a) acc += wx[a + rx] * row[ADJ ? a : -a];
        B[jb * TX + i] = acc;
    }
}

// y pass: v[e] at output row ty + 4 e.
// Forward: sum_b wy[b + ry] B[j + ry - b];  adjoint: B[j + ry + b].
template <typename T, bool ADJ>
__device__ __forceinline__ void ypass(const T *B, T (&v)[ROWS_PER_THREAD], const T *__restrict__ wy,
                                      int ry)
{
    const int i = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
#pragma unroll
    for (int e = 0; e < ROWS_PER_THREAD; ++e) {
        const int j = ty + (NT / TX) * e;
        const T *col = B + (j + ry) * TX + i;
        T acc = 0;
        for (int b = -ry; b <= ry; ++b) acc += wy[b + ry] * col[(ADJ ? b : -b) * TX];
        v[e] = acc;
    }
}

// Workgroup reduction of NV doubles (shuffle tree per wavefront, then the
// wavefronts in order); thread v < NV stores the total of value v to dst[v].
template <int NV>
__device__ __forceinline__ void wg_reduce_store(double (&q)[NV], double *red, double *dst)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = q[v];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[wave * NV + v] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NV + threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

// Iterate tile of slice k with a one-voxel halo into X ((TY+2) x (TX+2)).
template <typename T>
__device__ __forceinline__ void fill_x_tile(T *X, const T *__restrict__ x, const Geom &g, int k,
                                            int x0, int y0)
{
    const T *xs = x + (size_t)k * g.nx * g.ny;
    for (int e = threadIdx.x; e < XW * XH; e += NT) {
        const int jj = e / XW, ii = e - jj * XW;
        const int j = y0 - 1 + jj, i = x0 - 1 + ii;
        X[e] = (i >= 0 && i < g.nx && j >= 0 && j < g.ny) ? xs[(size_t)j * g.nx + i] : T(0);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Gradient pass.  For each output slice k of the segment:
//   (H^T r)_k = sum_c gz_{k+c}[c] XY^T_{k+c}(r_{k+c})
// computed by blurring every input slice m once (its own factors, adjoint
// form) and scattering it into the KZ pending outputs held in registers.
// Then, per mode:
//   GM_BLOCK: g = H^T r + lambda (VX^T w VX x + VY^T w VY x) + 2 eta (x - clip x)
//             + 2 kappa VZ^T VZ x, written to s.g, with <g,g>, <g,dp>, <dp,dp>;
//   GM_GRAD:  the same g written to out;
//   GM_EVAL:  no write; sums of ||g||^2, ||r||^2, TV, box and VZ terms of f;
//   GM_HT:    H^T r written to out.
// ---------------------------------------------------------------------------
template <typename T, int KZ>
__global__ void __launch_bounds__(NT)
k_grad(Geom g, Params prm, DevState<T> s, const T *__restrict__ rin, T *__restrict__ out,
       const Segment *__restrict__ segs, int mode, double *__restrict__ partials)
{
    constexpr int RZ = KZ / 2;
    __shared__ T A[LH * LW];
    __shared__ T B[LH * TX];
    __shared__ T X[XW * XH];
    __shared__ double red[(NT / 64) * NE];

    const Segment sg = segs[blockIdx.z];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int R = max(g.rx, g.ry);
    const int kx = 2 * g.rx + 1, ky = 2 * g.ry + 1;
    const size_t S = (size_t)g.nx * g.ny;
    const T lam = (T)prm.lambda, del2 = (T)(prm.delta * prm.delta), eta2 = (T)(2.0 * prm.eta),
            kap2 = (T)(2.0 * prm.kappa), lo = (T)prm.xmin, hi = (T)prm.xmax;
    const T *dpv = s.dp[sg.parity & 1];

    T acc[KZ][ROWS_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KZ; ++q)
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) acc[q][e] = 0;
    double qs[NE] = {0.0, 0.0, 0.0, 0.0, 0.0};

    for (int m = sg.z0 - RZ; m < sg.z0 + sg.n + RZ; ++m) {
        if (m >= 0 && m < g.nz) {
            const T *rs = rin + (size_t)m * S;
            __syncthreads();
            fill_halo(A, x0, y0, R, g, [&](int j, int i) { return rs[(size_t)j * g.nx + i]; });
            __syncthreads();
            xpass<T, true>(A, B, s.gx + (size_t)m * kx, g.rx, g.ry, R);
            __syncthreads();
            T v[ROWS_PER_THREAD];
            ypass<T, true>(B, v, s.gy + (size_t)m * ky, g.ry);
            const T *wz = s.gz + (size_t)m * KZ;
#pragma unroll
            for (int q = 0; q < KZ; ++q) {
                const T w = wz[2 * RZ - q];  // input m feeds output k = m - RZ + q with c = RZ - q
#pragma unroll
                for (int e = 0; e < ROWS_PER_THREAD; ++e) acc[q][e] += w * v[e];
            }
        }
        const int k = m - RZ;
        if (k >= sg.z0) {
            if (mode == GM_HT) {
#pragma unroll
                for (int e = 0; e < ROWS_PER_THREAD; ++e) {
                    const int j = y0 + ty + (NT / TX) * e, i = x0 + tx;
                    if (i < g.nx && j < g.ny) out[vidx(g, k, j, i)] = acc[0][e];
                }
            } else {
                __syncthreads();
                fill_x_tile(X, s.x, g, k, x0, y0);
                __syncthreads();
#pragma unroll
                for (int e = 0; e < ROWS_PER_THREAD; ++e) {
                    const int lj = ty + (NT / TX) * e, li = tx;
                    const int j = y0 + lj, i = x0 + li;
                    if (i >= g.nx || j >= g.ny) continue;
                    const T *xc = X + (lj + 1) * XW + (li + 1);
                    const T xv = xc[0];
                    const bool lastx = (i == g.nx - 1), lasty = (j == g.ny - 1);
                    // forward differences at (j,i), (j,i-1), (j-1,i)
                    const T dxc = lastx ? T(0) : xc[1] - xv;
                    const T dyc = lasty ? T(0) : xc[XW] - xv;
                    const T wc = T(1) / sqrt(dxc * dxc + dyc * dyc + del2);
                    T tv = -wc * (dxc + dyc);
                    if (i >= 1) {
                        const T dxl = xv - xc[-1];
                        const T dyl = lasty ? T(0) : xc[XW - 1] - xc[-1];
                        tv += dxl / sqrt(dxl * dxl + dyl * dyl + del2);
                    }
                    if (j >= 1) {
                        const T dxu = lastx ? T(0) : xc[-XW + 1] - xc[-XW];
                        const T dyu = xv - xc[-XW];
                        tv += dyu / sqrt(dxu * dxu + dyu * dyu + del2);
                    }
                    const T box = xv - clampv(xv, lo, hi);
                    T gv = acc[0][e] + lam * tv + eta2 * box;
                    T dz = 0;
                    if (prm.kappa != 0.0) {
                        const size_t o = vidx(g, k, j, i);
                        T zz = 0;
                        if (k >= 1) zz += xv - s.x[o - S];
                        if (k < g.nz - 1) {
                            dz = s.x[o + S] - xv;
                            zz -= dz;
                        }
                        gv += kap2 * zz;
                    }
                    const size_t o = vidx(g, k, j, i);
                    if (mode == GM_BLOCK) {
                        s.g[o] = gv;
                        const double gd = (double)gv, dd = (double)dpv[o];
                        qs[0] += gd * gd;
                        qs[1] += gd * dd;
                        qs[2] += dd * dd;
                    } else if (mode == GM_GRAD) {
                        out[o] = gv;
                    } else {  // GM_EVAL: terms of f in double
                        const double gd = (double)gv, rd = (double)rin[o];
                        const double dxd = (double)dxc, dyd = (double)dyc, dzd = (double)dz;
                        const double xd = (double)xv;
                        const double bx = xd - (xd < prm.xmin ? prm.xmin : (xd > prm.xmax ? prm.xmax : xd));
                        qs[0] += gd * gd;
                        qs[1] += rd * rd;
                        qs[2] += sqrt(dxd * dxd + dyd * dyd + prm.delta * prm.delta);
                        qs[3] += bx * bx;
                        qs[4] += dzd * dzd;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KZ - 1; ++q)
#pragma unroll
            for (int e = 0; e < ROWS_PER_THREAD; ++e) acc[q][e] = acc[q + 1][e];
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) acc[KZ - 1][e] = 0;
    }

    if (mode == GM_BLOCK || mode == GM_EVAL) {
        const size_t slot = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        if (mode == GM_BLOCK) {
            double q3[3] = {qs[0], qs[1], qs[2]};
            wg_reduce_store<3>(q3, red, partials + slot * NQ);
        } else {
            wg_reduce_store<NE>(qs, red, partials + slot * NE);
        }
    }
}

// ---------------------------------------------------------------------------
// Direction pass of a block S = [z0, z0+n): with d1 = -g and d2 = dp (both
// zero outside S), H d1 and H d2 on output slices S +- r_z:
//   (H d)_k = XY_k( sum_c gz_k[c] d_{k-c} )
// and the sums <Hd_a, Hd_b>, sum_S w (VX d_a VX d_b + VY d_a VY d_b) and
// <VZ d_a, VZ d_b> (a, b in {1, 2}) that fill the 2x2 majorant matrix.
// ---------------------------------------------------------------------------
template <typename T, int KZ>
__global__ void __launch_bounds__(NT)
k_dirs(Geom g, Params prm, DevState<T> s, const Segment *__restrict__ segs,
       double *__restrict__ partials)
{
    constexpr int RZ = KZ / 2;
    __shared__ T A1[LH * LW];
    __shared__ T A2[LH * LW];
    __shared__ T B1[LH * TX];
    __shared__ T B2[LH * TX];
    __shared__ double red[(NT / 64) * 9];

    const Segment sg = segs[blockIdx.z];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int R = max(g.rx, g.ry);
    const int kx = 2 * g.rx + 1, ky = 2 * g.ry + 1;
    const size_t S = (size_t)g.nx * g.ny;
    const T *__restrict__ gg = s.g;
    const T *__restrict__ dpv = s.dp[sg.parity & 1];
    const int z0 = sg.z0, z1 = sg.z0 + sg.n;
    const double del2 = prm.delta * prm.delta;

    double qs[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) qs[v] = 0.0;

    const int kb = max(0, z0 - max(RZ, 1)), ke = min(g.nz, z1 + RZ);
    for (int k = kb; k < ke; ++k) {
        const T *wz = s.gz + (size_t)k * KZ;
        __syncthreads();
        {
            const int w = TX + 2 * R, tot = w * (TY + 2 * R);
            for (int e = threadIdx.x; e < tot; e += NT) {
                const int jj = e / w, ii = e - jj * w;
                const int j = y0 - R + jj, i = x0 - R + ii;
                T v1 = 0, v2 = 0;
                if (i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
                    const size_t o = (size_t)j * g.nx + i;
#pragma unroll
                    for (int c = -RZ; c <= RZ; ++c) {
                        const int sl = k - c;
                        if (sl >= z0 && sl < z1) {
                            const T wv = wz[c + RZ];
                            v1 -= wv * gg[(size_t)sl * S + o];
                            v2 += wv * dpv[(size_t)sl * S + o];
                        }
                    }
                }
                A1[jj * LW + ii] = v1;
                A2[jj * LW + ii] = v2;
            }
        }
        __syncthreads();
        xpass<T, false>(A1, B1, s.gx + (size_t)k * kx, g.rx, g.ry, R);
        xpass<T, false>(A2, B2, s.gx + (size_t)k * kx, g.rx, g.ry, R);
        __syncthreads();
        T h1[ROWS_PER_THREAD], h2[ROWS_PER_THREAD];
        ypass<T, false>(B1, h1, s.gy + (size_t)k * ky, g.ry);
        ypass<T, false>(B2, h2, s.gy + (size_t)k * ky, g.ry);
        const bool ink = (k >= z0 && k < z1);
        const bool zterm = (prm.kappa != 0.0) && k >= z0 - 1 && k < z1 && k < g.nz - 1;
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) {
            const int j = y0 + ty + (NT / TX) * e, i = x0 + tx;
            if (i >= g.nx || j >= g.ny) continue;
            const double a = (double)h1[e], b = (double)h2[e];
            qs[0] += a * a;
            qs[1] += a * b;
            qs[2] += b * b;
            const size_t o = vidx(g, k, j, i);
            if (ink) {
                const bool lastx = (i == g.nx - 1), lasty = (j == g.ny - 1);
                const double xv = (double)s.x[o];
                const double dxx = lastx ? 0.0 : (double)s.x[o + 1] - xv;
                const double dyx = lasty ? 0.0 : (double)s.x[o + g.nx] - xv;
                const double w = 1.0 / sqrt(dxx * dxx + dyx * dyx + del2);
                const double g0 = (double)gg[o], p0 = (double)dpv[o];
                const double dx1 = lastx ? 0.0 : g0 - (double)gg[o + 1];
                const double dy1 = lasty ? 0.0 : g0 - (double)gg[o + g.nx];
                const double dx2 = lastx ? 0.0 : (double)dpv[o + 1] - p0;
                const double dy2 = lasty ? 0.0 : (double)dpv[o + g.nx] - p0;
                qs[3] += w * (dx1 * dx1 + dy1 * dy1);
                qs[4] += w * (dx1 * dx2 + dy1 * dy2);
                qs[5] += w * (dx2 * dx2 + dy2 * dy2);
            }
            if (zterm) {
                // VZ d at slice k: d_{k+1} - d_k with d zero outside S
                double z1v = 0.0, z2v = 0.0;
                if (k + 1 >= z0 && k + 1 < z1) {
                    z1v -= (double)gg[o + S];
                    z2v += (double)dpv[o + S];
                }
                if (ink) {
                    z1v += (double)gg[o];
                    z2v -= (double)dpv[o];
                }
                qs[6] += z1v * z1v;
                qs[7] += z1v * z2v;
                qs[8] += z2v * z2v;
            }
        }
    }
    const size_t slot = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    wg_reduce_store<9>(qs, red, partials + slot * NQ + 3);
}

// ---------------------------------------------------------------------------
// Update pass of a block S: d' = u1 d1 + u2 d2 = -u1 g + u2 dp on S;
// r += H d' on S +- r_z; x_S += d'; dp_out,S = d'.  The previous step is
// read from dp[parity] and written to dp[parity ^ 1], so workgroups reading
// a neighbour's halo never see a half-updated step.
// ---------------------------------------------------------------------------
template <typename T, int KZ>
__global__ void __launch_bounds__(NT)
k_update(Geom g, DevState<T> s, const Segment *__restrict__ segs, const double *__restrict__ u)
{
    constexpr int RZ = KZ / 2;
    __shared__ T A[LH * LW];
    __shared__ T B[LH * TX];

    const Segment sg = segs[blockIdx.z];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int R = max(g.rx, g.ry);
    const int kx = 2 * g.rx + 1, ky = 2 * g.ry + 1;
    const size_t S = (size_t)g.nx * g.ny;
    const T u1 = (T)u[2 * sg.block], u2 = (T)u[2 * sg.block + 1];
    const T *__restrict__ gg = s.g;
    const T *__restrict__ dpi = s.dp[sg.parity & 1];
    T *__restrict__ dpo = s.dp[(sg.parity & 1) ^ 1];
    const int z0 = sg.z0, z1 = sg.z0 + sg.n;

    const int kb = max(0, z0 - RZ), ke = min(g.nz, z1 + RZ);
    for (int k = kb; k < ke; ++k) {
        const T *wz = s.gz + (size_t)k * KZ;
        __syncthreads();
        fill_halo(A, x0, y0, R, g, [&](int j, int i) {
            const size_t o = (size_t)j * g.nx + i;
            T v = 0;
#pragma unroll
            for (int c = -RZ; c <= RZ; ++c) {
                const int sl = k - c;
                if (sl >= z0 && sl < z1) {
                    const size_t q = (size_t)sl * S + o;
                    const T d = u2 * dpi[q] - u1 * gg[q];
                    v += wz[c + RZ] * d;
                }
            }
            return v;
        });
        __syncthreads();
        xpass<T, false>(A, B, s.gx + (size_t)k * kx, g.rx, g.ry, R);
        __syncthreads();
        T h[ROWS_PER_THREAD];
        ypass<T, false>(B, h, s.gy + (size_t)k * ky, g.ry);
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) {
            const int j = y0 + ty + (NT / TX) * e, i = x0 + tx;
            if (i < g.nx && j < g.ny) s.r[vidx(g, k, j, i)] += h[e];
        }
    }
    for (int k = z0; k < z1; ++k) {
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) {
            const int j = y0 + ty + (NT / TX) * e, i = x0 + tx;
            if (i >= g.nx || j >= g.ny) continue;
            const size_t q = vidx(g, k, j, i);
            const T d = u2 * dpi[q] - u1 * gg[q];
            s.x[q] += d;
            dpo[q] = d;
        }
    }
}

// ---------------------------------------------------------------------------
// out = H(in) - sub on the slices of each segment (sub may be null).
// ---------------------------------------------------------------------------
template <typename T, int KZ>
__global__ void __launch_bounds__(NT)
k_H(Geom g, DevState<T> s, const T *__restrict__ in, const T *__restrict__ sub,
    T *__restrict__ out, const Segment *__restrict__ segs)
{
    constexpr int RZ = KZ / 2;
    __shared__ T A[LH * LW];
    __shared__ T B[LH * TX];
    const Segment sg = segs[blockIdx.z];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int R = max(g.rx, g.ry);
    const int kx = 2 * g.rx + 1, ky = 2 * g.ry + 1;
    const size_t S = (size_t)g.nx * g.ny;
    for (int k = sg.z0; k < sg.z0 + sg.n; ++k) {
        const T *wz = s.gz + (size_t)k * KZ;
        __syncthreads();
        fill_halo(A, x0, y0, R, g, [&](int j, int i) {
            const size_t o = (size_t)j * g.nx + i;
            T v = 0;
#pragma unroll
            for (int c = -RZ; c <= RZ; ++c) {
                const int sl = k - c;
                if (sl >= 0 && sl < g.nz) v += wz[c + RZ] * in[(size_t)sl * S + o];
            }
            return v;
        });
        __syncthreads();
        xpass<T, false>(A, B, s.gx + (size_t)k * kx, g.rx, g.ry, R);
        __syncthreads();
        T h[ROWS_PER_THREAD];
        ypass<T, false>(B, h, s.gy + (size_t)k * ky, g.ry);
#pragma unroll
        for (int e = 0; e < ROWS_PER_THREAD; ++e) {
            const int j = y0 + ty + (NT / TX) * e, i = x0 + tx;
            if (i < g.nx && j < g.ny) {
                const size_t o = vidx(g, k, j, i);
                out[o] = sub ? h[e] - sub[o] : h[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per block: fixed-order reduction of its slots, then the 2x2 system of the
// memory-gradient subspace (Sec. 2.3, eq. "minimizer"):
//   B = D^T A_S D with D = [d1 | d2], d1 = -g, d2 = dp,
//   c = D^T g = (-<g,g>, <dp,g>),  u = -B^+ c.
// B^+ is the exact inverse when det > 1e-12 B11 B22, else the rank-one
// pseudo-inverse B / tr(B)^2 (zero when tr(B) = 0).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT)
k_solve(Params prm, const Segment *__restrict__ segs, int slots, const double *__restrict__ partials,
        double *__restrict__ u, double *__restrict__ info)
{
    __shared__ double red[NT];
    __shared__ double tot[NQ];
    const Segment sg = segs[blockIdx.x];
    const double *p = partials + (size_t)blockIdx.x * slots * NQ;
    for (int v = 0; v < NQ; ++v) {
        double s = 0.0;
        for (int t = threadIdx.x; t < slots; t += NT) s += p[(size_t)t * NQ + v];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot[v] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gg = tot[0], gd = tot[1], dd = tot[2];
        const double e2 = 2.0 * prm.eta, k2 = 2.0 * prm.kappa, lam = prm.lambda;
        const double b11 = tot[3] + e2 * gg + lam * tot[6] + k2 * tot[9];
        const double b12 = tot[4] - e2 * gd + lam * tot[7] + k2 * tot[10];
        const double b22 = tot[5] + e2 * dd + lam * tot[8] + k2 * tot[11];
        const double c1 = -gg, c2 = gd;
        const double det = b11 * b22 - b12 * b12, tr = b11 + b22;
        double p11, p12, p22;
        if (det > 1e-12 * b11 * b22) {
            p11 = b22 / det;
            p12 = -b12 / det;
            p22 = b11 / det;
        } else if (tr > 0.0) {
            const double t2 = tr * tr;
            p11 = b11 / t2;
            p12 = b12 / t2;
            p22 = b22 / t2;
        } else {
            p11 = p12 = p22 = 0.0;
        }
        const double u1 = -(p11 * c1 + p12 * c2);
        const double u2 = -(p12 * c1 + p22 * c2);
        u[2 * sg.block] = u1;
        u[2 * sg.block + 1] = u2;
        if (info) {
            double *o = info + 8 * sg.block;
            o[0] = b11; o[1] = b12; o[2] = b22; o[3] = c1; o[4] = c2; o[5] = u1; o[6] = u2; o[7] = gg;
        }
    }
}

__global__ void __launch_bounds__(NT)
k_sum_eval(const double *__restrict__ partials, int nslot, double *__restrict__ out)
{
    __shared__ double red[NT];
    for (int v = 0; v < NE; ++v) {
        double s = 0.0;
        for (int t = threadIdx.x; t < nslot; t += NT) s += partials[(size_t)t * NE + v];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = red[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers: dispatch on the z extent of the PSF (a template parameter so the
// ring and the z-combine unroll).
// ---------------------------------------------------------------------------
#define BD3MG_KZ_SWITCH(kz, CALL)          \
    switch (kz) {                          \
    case 1: { constexpr int KZ = 1; CALL; } break; \
    case 3: { constexpr int KZ = 3; CALL; } break; \
    case 5: { constexpr int KZ = 5; CALL; } break; \
    case 7: { constexpr int KZ = 7; CALL; } break; \
    case 9: { constexpr int KZ = 9; CALL; } break; \
    default: return hipErrorInvalidValue;  \
    }

static dim3 grid_of(const Geom &g, int nseg) { return dim3(g.ntx, g.nty, nseg); }

template <typename T>
hipError_t launch_grad(const Geom &g, const Params &prm, const DevState<T> &s, const T *rin, T *out,
                       const Segment *segs, int nseg, int mode, double *partials, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1,
                    hipLaunchKernelGGL((k_grad<T, KZ>), grid_of(g, nseg), dim3(NT), 0, st, g, prm,
                                       s, rin, out, segs, mode, partials));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dirs(const Geom &g, const Params &prm, const DevState<T> &s, const Segment *segs,
                       int nseg, double *partials, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1,
                    hipLaunchKernelGGL((k_dirs<T, KZ>), grid_of(g, nseg), dim3(NT), 0, st, g, prm,
                                       s, segs, partials));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Geom &g, const DevState<T> &s, const Segment *segs, int nseg,
                         const double *u, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1,
                    hipLaunchKernelGGL((k_update<T, KZ>), grid_of(g, nseg), dim3(NT), 0, st, g, s,
                                       segs, u));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_H(const Geom &g, const DevState<T> &s, const T *in, const T *sub, T *out,
                    const Segment *segs, int nseg, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1,
                    hipLaunchKernelGGL((k_H<T, KZ>), grid_of(g, nseg), dim3(NT), 0, st, g, s, in,
                                       sub, out, segs));
    return hipGetLastError();
}

hipError_t launch_solve(const Params &prm, const Segment *segs, int nseg, int slots_per_seg,
                        const double *partials, double *u, double *info, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve, dim3(nseg), dim3(NT), 0, st, prm, segs, slots_per_seg, partials, u,
                       info);
    return hipGetLastError();
}

hipError_t launch_sum_eval(const double *partials, int nslot, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_eval, dim3(1), dim3(NT), 0, st, partials, nslot, out);
    return hipGetLastError();
}

// Streaming copy, 16 bytes per lane per iteration, grid-stride.
__global__ void __launch_bounds__(NT) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                             size_t n)
{
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, size_t n16, hipStream_t st)
{
    // 256 CUs x 8 workgroups keep every CU streaming
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(NT), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

#define BD3MG_INSTANTIATE(T)                                                                     \
    template hipError_t launch_grad<T>(const Geom &, const Params &, const DevState<T> &,         \
                                       const T *, T *, const Segment *, int, int, double *,      \
                                       hipStream_t);                                             \
    template hipError_t launch_dirs<T>(const Geom &, const Params &, const DevState<T> &,         \
                                       const Segment *, int, double *, hipStream_t);             \
    template hipError_t launch_update<T>(const Geom &, const DevState<T> &, const Segment *, int, \
                                         const double *, hipStream_t);                           \
    template hipError_t launch_H<T>(const Geom &, const DevState<T> &, const T *, const T *, T *, \
                                    const Segment *, int, hipStream_t);

BD3MG_INSTANTIATE(float)
BD3MG_INSTANTIATE(double)

}  // namespace bd3mg
