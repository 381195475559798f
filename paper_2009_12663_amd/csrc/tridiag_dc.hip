// Eigenpairs of the symmetric tridiagonal T (diagonal d, off-diagonal e, e[i] =
// T(i, i+1)) from the Householder reduction of Omega, for Alg. 3's small symmetric
// eigenproblem (Omega = U_s Lambda U_s^T), by divide and conquer (Cuppen 1981):
//
//   T = diag(T_A - b e_last e_last^T, T_B - b e_1 e_1^T) + b u u^T,  u = e_last + e_1,
//
// so with T_A = Q_A D_A Q_A^T and T_B = Q_B D_B Q_B^T the merged problem is
// diag(D_A, D_B) + rho z z^T with rho = 2 b and z = [Q_A's last row, Q_B's first row]
// / sqrt 2.  Its eigenvalues are the roots of the secular equation
// f(x) = 1 + rho sum_i z_i^2 / (d_i - x), one between consecutive poles and one above
// the last (rho > 0; a negative rho is handled by negating D).  Steps of a merge:
//   * sort the poles; deflate components with |rho z_i| <= tol, and close poles by a
//     Givens rotation that moves one pole's weight onto its neighbour;
//   * each root by safeguarded Newton steps on tau f(tau) inside a bracket that every
//     evaluation's sign narrows (falling back to the bracket's midpoint), measured from
//     the nearer pole (x = d_o + tau), so that differences x - d_i keep their relative
//     accuracy;
//   * z recomputed from the roots (Loewner's formula; Gu and Eisenstat 1994), which
//     makes the eigenvectors z_i / (d_i - x_j) numerically orthogonal;
//   * the merged basis: the sorted, rotated columns of diag(Q_A, Q_B) times those
//     eigenvectors.
// The merges run bottom-up over power-of-two blocks (leaf i starts at d_i - e_{i-1}
// - e_i, since every adjacent pair is split at some level), one workgroup per merge,
// all merges of a level in one launch.  Z = Q_H Y then gives the eigenvectors of Omega.
#include <cmath>

#include "common.h"

namespace {

constexpr double EPS = 2.220446049250313e-16;   // 2^-52
constexpr int DC_MAX = 256;
constexpr int DC_THREADS = 256;

// Leaves: lam_i = d_i - e_{i-1} - e_i, Q = I.
__global__ void dc_leaves(int c, const double* __restrict__ d, const double* __restrict__ e, double* __restrict__ lam,
                          double* __restrict__ Q, int32_t* __restrict__ status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c * c; i += gridDim.x * blockDim.x) {
        const int col = i / c, row = i % c;
        Q[i] = col == row ? 1.0 : 0.0;
        if (row == 0) {
            const double el = col > 0 ? e[col - 1] : 0.0, er = col + 1 < c ? e[col] : 0.0;
            const double v = d[col] - el - er;
            lam[col] = v;
            if (!isfinite(d[col]) || !isfinite(el) || !isfinite(er)) set_status(status, BFGS_ERR_NUMERIC);
        }
    }
}

// One merge of blocks [s, s + h) and [s + h, s + h + hb) per workgroup.  Qin/lam_in hold
// the blocks' eigenvectors (block-diagonal, column-major c x c) and eigenvalues;
// Qout/lam_out receive the merged ones.  R and U are c x c scratch (block regions).
__global__ void __launch_bounds__(DC_THREADS) dc_merge(int c, int h, const double* __restrict__ e,
                                                       const double* __restrict__ lam_in, const double* __restrict__ Qin,
                                                       double* __restrict__ lam_out, double* __restrict__ Qout,
                                                       double* __restrict__ R, double* __restrict__ U,
                                                       int* __restrict__ Kg, int* __restrict__ ndx_g,
                                                       int* __restrict__ slot_g) {
    __shared__ double Dv[DC_MAX], zv[DC_MAX], ds[DC_MAX], zs[DC_MAX];
    __shared__ int pcol[DC_MAX], ndx[DC_MAX], slot_of[DC_MAX];
    __shared__ unsigned char defl[DC_MAX];
    __shared__ double dn[DC_MAX], z2n[DC_MAX], zn[DC_MAX], taun[DC_MAX], zh[DC_MAX], lamn[DC_MAX];
    __shared__ int orgn[DC_MAX];
    __shared__ int rot_a[DC_MAX], rot_b[DC_MAX];
    __shared__ double rot_c[DC_MAX], rot_s[DC_MAX];
    __shared__ int nrot_sh, K_sh;
    const int tid = threadIdx.x;
    const int s = blockIdx.x * 2 * h;
    if (s >= c) return;                                   // whole workgroup
    const int ha = min(h, c - s);
    const int hb = min(h, c - s - ha);
    const int n = ha + hb;
    if (hb == 0) {
        // nothing to merge: copy the block (dc_merge_gemm skips it)
        if (tid == 0) Kg[blockIdx.x] = -1;
        for (int t = tid; t < n * n; t += DC_THREADS) {
            const int col = s + t / n, row = s + t % n;
            Qout[(int64_t)col * c + row] = Qin[(int64_t)col * c + row];
        }
        for (int t = tid; t < n; t += DC_THREADS) lam_out[s + t] = lam_in[s + t];
        return;
    }
    const double beta = e[s + ha - 1];
    const bool neg = beta < 0.0;
    const double rho = 2.0 * fabs(beta);
    const double r2 = 0.7071067811865476;   // 1 / sqrt 2
    // poles and weights (negated when beta < 0, so that rho > 0)
    for (int t = tid; t < n; t += DC_THREADS) {
        const double dv = lam_in[s + t];
        Dv[t] = neg ? -dv : dv;
        zv[t] = r2 * (t < ha ? Qin[(int64_t)(s + t) * c + s + ha - 1] : Qin[(int64_t)(s + t) * c + s + ha]);
    }
    __syncthreads();
    // sort by rank (ties by index).  The order is total even for NaN (after every
    // number, among themselves by index), so the ranks are a permutation and every
    // pcol entry is written: a non-finite input gives wrong values, never an index
    // out of range.
    for (int t = tid; t < n; t += DC_THREADS) {
        const double dt = Dv[t];
        const bool nt = isnan(dt);
        int rk = 0;
        for (int u = 0; u < n; ++u) {
            const double du = Dv[u];
            const bool before = isnan(du) ? (nt && u < t) : (nt || du < dt || (du == dt && u < t));
            rk += before ? 1 : 0;
        }
        ds[rk] = dt;
        zs[rk] = zv[t];
        pcol[rk] = t;
    }
    __syncthreads();
    // deflation scan (one lane)
    if (tid == 0) {
        double dmax = rho;
        for (int p = 0; p < n; ++p) dmax = fmax(dmax, fabs(ds[p]));
        const double tol = 8.0 * EPS * dmax;
        int nrot = 0, last = -1, K = 0;
        for (int p = 0; p < n; ++p) {
            defl[p] = fabs(rho * zs[p]) <= tol ? 1 : 0;
            if (defl[p]) continue;
            if (last >= 0) {
                const double zl = zs[last], zi = zs[p];
                const double tau = sqrt(fma(zl, zl, zi * zi));
                const double cc = zi / tau, sn = -zl / tau;
                if (fabs((ds[p] - ds[last]) * cc * sn) <= tol) {
                    zs[p] = tau;
                    zs[last] = 0.0;
                    const double dl = ds[last], di = ds[p];
                    ds[last] = dl * cc * cc + di * sn * sn;
                    ds[p] = dl * sn * sn + di * cc * cc;
                    defl[last] = 1;
                    rot_a[nrot] = last;
                    rot_b[nrot] = p;
                    rot_c[nrot] = cc;
                    rot_s[nrot] = sn;
                    ++nrot;
                }
            }
            last = p;
        }
        for (int p = 0; p < n; ++p) {
            if (!defl[p]) {
                ndx[K] = p;
                slot_of[p] = K;
                ++K;
            } else {
                slot_of[p] = -1;
            }
        }
        nrot_sh = nrot;
        K_sh = K;
    }
    __syncthreads();
    const int K = K_sh, nrot = nrot_sh;
    for (int j = tid; j < K; j += DC_THREADS) {
        const double zj = zs[ndx[j]];
        dn[j] = ds[ndx[j]];
        zn[j] = zj;
        z2n[j] = zj * zj;
    }
    __syncthreads();
    // secular roots: lane j finds root j from its nearer pole (bracket, then Newton)
    double z2sum = 0.0;
    for (int i = 0; i < K; ++i) z2sum += z2n[i];
    for (int j = tid; j < K; j += DC_THREADS) {
        int o;
        double a, b;
        if (j < K - 1) {
            const double mid = 0.5 * (dn[j] + dn[j + 1]);
            double f = 1.0;
            for (int i = 0; i < K; ++i) f += rho * z2n[i] / (dn[i] - mid);
            if (f > 0.0) {
                o = j;
                a = 0.0;
                b = mid - dn[j];
            } else {
                o = j + 1;
                a = mid - dn[j + 1];
                b = 0.0;
            }
        } else {
            o = K - 1;
            a = 0.0;
            b = rho * z2sum;
        }
        // Newton on h(t) = t f(t), which has the same root but no pole at the origin
        // (that term of t f is the constant -rho z_o^2; the other pole is at least twice
        // as far as the root).  The iterate stays inside the bracket [a, b] that each
        // evaluation's sign of f narrows (f increases in t); a step that leaves it is
        // replaced by the bracket's midpoint.
        const double dorg = dn[o];
        double t = 0.5 * (a + b);
        for (int it = 0; it < 256; ++it) {
            double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
            int i = 0;
            for (; i + 4 <= K; i += 4) {
                const double q0 = 1.0 / ((dn[i] - dorg) - t), q1 = 1.0 / ((dn[i + 1] - dorg) - t);
                const double q2 = 1.0 / ((dn[i + 2] - dorg) - t), q3 = 1.0 / ((dn[i + 3] - dorg) - t);
                const double w0 = z2n[i] * q0, w1 = z2n[i + 1] * q1, w2 = z2n[i + 2] * q2, w3 = z2n[i + 3] * q3;
                f0 += w0;
                f1 += w1;
                f2 += w2;
                f3 += w3;
                g0 = fma(w0, q0, g0);
                g1 = fma(w1, q1, g1);
                g2 = fma(w2, q2, g2);
                g3 = fma(w3, q3, g3);
            }
            for (; i < K; ++i) {
                const double q = 1.0 / ((dn[i] - dorg) - t), w = z2n[i] * q;
                f0 += w;
                g0 = fma(w, q, g0);
            }
            const double f = fma(rho, (f0 + f1) + (f2 + f3), 1.0);
            const double fp = rho * ((g0 + g1) + (g2 + g3));
            if (f == 0.0) break;
            if (f > 0.0) b = t;
            else a = t;
            const double step = t * f / fma(t, fp, f);
            double tn = t - step;
            if (fabs(step) <= 2.0 * EPS * fabs(t)) {
                t = tn;
                break;
            }
            if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
            t = tn;
            if (b - a <= 2.0 * EPS * fmax(fabs(a), fabs(b))) break;
        }
        orgn[j] = o;
        taun[j] = t;
        lamn[j] = dorg + t;
    }
    __syncthreads();
    // Loewner: zh_i^2 = prod_j (x_j - d_i) / prod_{j != i} (d_j - d_i) / rho
    for (int i = tid; i < K; i += DC_THREADS) {
        const double di = dn[i];
        double p = (dn[orgn[K - 1]] - di) + taun[K - 1];
        for (int j = 0; j < K - 1; ++j) {
            const double lj = (dn[orgn[j]] - di) + taun[j];
            const double dd = j >= i ? dn[j + 1] - di : dn[j] - di;
            p *= lj / dd;
        }
        p /= rho;
        zh[i] = copysign(sqrt(fmax(p, 0.0)), zn[i]);
    }
    __syncthreads();
    // U (K x K, column j = normalised zh / (d - x_j)) in the block region of U
    for (int j = tid; j < K; j += DC_THREADS) {
        double ss = 0.0;
        for (int i = 0; i < K; ++i) {
            const double v = zh[i] / ((dn[i] - dn[orgn[j]]) - taun[j]);
            ss = fma(v, v, ss);
        }
        const double inv = 1.0 / sqrt(ss);
        for (int i = 0; i < K; ++i) U[(int64_t)(s + j) * c + s + i] = zh[i] / ((dn[i] - dn[orgn[j]]) - taun[j]) * inv;
    }
    // rotated basis R: row r, sorted column p = column pcol[p] of diag(Q_A, Q_B) (only the
    // diagonal blocks of Qin are current; the rest is zero), then the deflation
    // rotations in order (one thread per row)
    for (int r = tid; r < n; r += DC_THREADS) {
        double* Rr = R + s + r;   // R[(s + p) * c + s + r]
        for (int p = 0; p < n; ++p) {
            const int q = pcol[p];
            Rr[(int64_t)(s + p) * c] = (q < ha) == (r < ha) ? Qin[(int64_t)(s + q) * c + s + r] : 0.0;
        }
        for (int q = 0; q < nrot; ++q) {
            const int pa = rot_a[q], pb = rot_b[q];
            const double cc = rot_c[q], sn = rot_s[q];
            const double xa = Rr[(int64_t)(s + pa) * c], xb = Rr[(int64_t)(s + pb) * c];
            Rr[(int64_t)(s + pa) * c] = cc * xa + sn * xb;
            Rr[(int64_t)(s + pb) * c] = -sn * xa + cc * xb;
        }
    }
    // the merged basis (R[:, ndx] U, deflated columns as rotated) is formed by dc_merge_gemm
    if (tid == 0) Kg[blockIdx.x] = K;
    for (int p = tid; p < n; p += DC_THREADS) {
        slot_g[s + p] = slot_of[p];
        ndx_g[s + p] = p < K ? ndx[p] : 0;
    }
    for (int p = tid; p < n; p += DC_THREADS) {
        const int j = slot_of[p];
        const double v = j < 0 ? ds[p] : lamn[j];
        lam_out[s + p] = neg ? -v : v;
    }
}

// Merged basis of each merge of the level: column p of the block is R[:, p] when p was
// deflated, else R[:, ndx] U[:, slot(p)].  Grid (merges, tiles of 64 x 64 outputs);
// thread = 4 x 4 outputs; the reduction is staged 16 deep in LDS.
constexpr int MG_T = 64, MG_K = 16;

__global__ void __launch_bounds__(256) dc_merge_gemm(int c, int h, const double* __restrict__ R,
                                                     const double* __restrict__ U, const int* __restrict__ Kg,
                                                     const int* __restrict__ ndx_g, const int* __restrict__ slot_g,
                                                     double* __restrict__ Qout) {
    __shared__ double As[MG_K][MG_T + 1];   // As[k][r] = R(r, ndx[k])
    __shared__ double Bs[MG_K][MG_T + 1];   // Bs[k][p] = U(k, slot(p))
    const int b = blockIdx.x, K = Kg[b];
    if (K < 0) return;                      // whole workgroup: block copied by dc_merge
    const int s = b * 2 * h, n = min(2 * h, c - s);
    const int tpd = (2 * h + MG_T - 1) / MG_T;
    const int r0 = (blockIdx.y / tpd) * MG_T, p0 = (blockIdx.y % tpd) * MG_T;
    if (r0 >= n || p0 >= n) return;         // whole workgroup
    const int tid = threadIdx.x, tr = tid / 16, tp = tid % 16;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += MG_K) {
        for (int e = tid; e < MG_K * MG_T; e += 256) {
            const int kk = e / MG_T, rr = e % MG_T, k = k0 + kk;
            As[kk][rr] = (k < K && r0 + rr < n) ? R[(int64_t)(s + ndx_g[s + k]) * c + s + r0 + rr] : 0.0;
            const int pp = e % MG_T, kb = e / MG_T, kq = k0 + kb;
            int j = p0 + pp < n ? slot_g[s + p0 + pp] : -1;
            Bs[kb][pp] = (kq < K && j >= 0) ? U[(int64_t)(s + j) * c + s + kq] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < MG_K; ++kk) {
            double a[4], bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][tr * 4 + u];
                bb[u] = Bs[kk][tp * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], bb[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int p = p0 + tp * 4 + v;
        if (p >= n) continue;
        const bool defl = slot_g[s + p] < 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + tr * 4 + u;
            if (r < n) Qout[(int64_t)(s + p) * c + s + r] = defl ? R[(int64_t)(s + p) * c + s + r] : acc[u][v];
        }
    }
}

// C = A B, all c x c column-major; block (ceil(c / 64), c): lane -> row, y -> column.
__global__ void __launch_bounds__(64) dc_gemm_nn(int c, const double* __restrict__ A, const double* __restrict__ B,
                                                 double* __restrict__ C) {
    const int r = blockIdx.x * 64 + threadIdx.x, col = blockIdx.y;
    if (r >= c) return;
    const double* bc = B + (int64_t)col * c;
    double acc = 0.0;
    for (int k = 0; k < c; ++k) acc = fma(A[(int64_t)k * c + r], bc[k], acc);
    C[(int64_t)col * c + r] = acc;
}

}  // namespace

size_t tridiag_dc_workspace(int c) { return ((size_t)4 * c * c + 2 * (size_t)c) * sizeof(double) + (size_t)4 * c * sizeof(int); }

int tridiag_dc(hipStream_t st, int c, const double* d, const double* e, const double* Qh, double* work, double** w_out,
               double* Z, int32_t* status) {
    if (c < 1 || c > DC_MAX) return BFGS_ERR_ARG;
    const size_t cc = (size_t)c * c;
    double* Qa = work;
    double* Qb = Qa + cc;
    double* R = Qb + cc;
    double* U = R + cc;
    double* la = U + cc;
    double* lb = la + c;
    int* Kg = (int*)(lb + c);
    int* ndx_g = Kg + c;
    int* slot_g = ndx_g + c;
    hipLaunchKernelGGL(dc_leaves, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, st, c, d, e, la, Qa, status);
    for (int h = 1; h < c; h *= 2) {
        const int nb = ceil_div(c, 2 * h);
        const int tpd = ceil_div(2 * h, MG_T);
        hipLaunchKernelGGL(dc_merge, dim3(nb), dim3(DC_THREADS), 0, st, c, h, e, la, Qa, lb, Qb, R, U, Kg, ndx_g,
                           slot_g);
        hipLaunchKernelGGL(dc_merge_gemm, dim3(nb, tpd * tpd), dim3(256), 0, st, c, h, R, U, Kg, ndx_g, slot_g, Qb);
        std::swap(Qa, Qb);
        std::swap(la, lb);
    }
    hipLaunchKernelGGL(dc_gemm_nn, dim3(ceil_div(c, 64), c), dim3(64), 0, st, c, Qh, Qa, Z);
    *w_out = la;
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}
