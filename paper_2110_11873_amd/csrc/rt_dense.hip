// rt_dense.hip -- kernels on the assembled A: the SOR and SSOR preconditioners
// (Sect. 2.3) and their product form.
//
// With A = D + L + U (diagonal, strict lower and upper triangles in the
// unknowns' order) the preconditioners are
//   SOR   P = omega^-1 D + U,
//   SSOR  P = omega (2 - omega)^-1 (omega^-1 D + U) D^-1 (omega^-1 D + L).
// One workgroup per slab keeps the slab's vector (at most 2 RT_MAX_NS values)
// in LDS and walks the triangle in blocks of 64 unknowns: the block's
// diagonal 64 x 64 part is staged in LDS and solved by one wavefront, the
// solved values are broadcast with readlane, and the rows still to come are
// updated with the block's columns (16 lanes per row, each row's 64 entries
// read once, contiguously).  Each triangle of A is read from memory once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kTriNT = 256;
constexpr int kTriPass = 4;  // 16-row passes of the update loaded together
constexpr int kTriB = 64;
constexpr int kTriPad = kTriB + 1;  // padded row of the staged block

__device__ inline double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// r <- (omega^-1 D + T)^-1 r for T the strict upper (UP) or lower triangle
// of the slab's A (row-major, N x N), r in LDS; UNIT: a unit diagonal instead
// of omega^-1 D (the L factor of an LU factorization).
template <bool UP, bool UNIT = false, bool ROWWISE = false>
__device__ void tri_sweep(const double *A, int N, double om, double *r, double *blk) {
    const int tid = threadIdx.x;
    const int nb = (N + kTriB - 1) / kTriB;
    constexpr int kStage = kTriB * kTriB / kTriNT;
    // a block's diagonal part, loaded into registers (all loads in flight
    // together); the next block's is loaded before this block's update
    auto load_diag = [&](int b, double *stage) {
        const int i0 = b * kTriB, n = min(kTriB, N - i0);
#pragma unroll
        for (int t = 0; t < kStage; ++t) {
            const int e = tid + t * kTriNT, rr = e / kTriB, cc = e % kTriB;
            stage[t] = (rr < n && cc < n) ? A[(long long)(i0 + rr) * N + i0 + cc] : 0.0;
        }
    };
    double stage[kStage];
    if constexpr (!ROWWISE) load_diag(UP ? nb - 1 : 0, stage);
    for (int bi = 0; bi < nb; ++bi) {
        const int b = UP ? nb - 1 - bi : bi;
        const int i0 = b * kTriB, n = min(kTriB, N - i0);
        if constexpr (ROWWISE) load_diag(b, stage);  // no registers to spare during the update
#pragma unroll
        for (int t = 0; t < kStage; ++t) {
            const int e = tid + t * kTriNT;
            blk[(e / kTriB) * kTriPad + e % kTriB] = stage[t];
        }
        __syncthreads();
        if constexpr (!ROWWISE)
            if (bi + 1 < nb) load_diag(UP ? b - 1 : b + 1, stage);
        if (tid < kWave) {
            const int c = tid;
            double val = c < n ? r[i0 + c] : 0.0;
            const double dc = c < n ? (UNIT ? 1.0 : om / blk[c * kTriPad + c]) : 0.0;
            if (n == kTriB) {
                // a full block: eight steps at a time, their LDS reads issued first
                // (the outer loop stays rolled: one group's reads in registers)
#pragma unroll 1
                for (int i8 = 0; i8 < kTriB; i8 += 8) {
                    double col[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = UP ? kTriB - 1 - (i8 + u) : i8 + u;
                        col[u] = blk[c * kTriPad + i];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = UP ? kTriB - 1 - (i8 + u) : i8 + u;
                        const double zi = readlane_d(val * dc, i);
                        if (c == i) val = zi;
                        else if (UP ? c < i : c > i) val -= col[u] * zi;
                    }
                }
            } else {
                for (int ii = 0; ii < n; ++ii) {
                    const int i = UP ? n - 1 - ii : ii;
                    const double zi = readlane_d(val * dc, i);
                    if (c == i) val = zi;
                    else if (UP ? c < i : c > i) val -= blk[c * kTriPad + i] * zi;
                }
            }
            if (c < n) r[i0 + c] = val;
        }
        __syncthreads();
        const int lo = UP ? 0 : i0 + n, hi = UP ? i0 : N;
        if constexpr (ROWWISE) {
            // one thread per row, each row's 64 entries loaded together: the
            // most bytes in flight per thread (a lone large slab)
            for (int l = lo + tid; l < hi; l += kTriNT) {
                const double2 *row = reinterpret_cast<const double2 *>(A + (long long)l * N + i0);
                double acc0 = 0.0, acc1 = 0.0;
                if (n == kTriB) {
                    double2 v[kTriB / 2];
#pragma unroll
                    for (int c2 = 0; c2 < kTriB / 2; ++c2) v[c2] = row[c2];
#pragma unroll
                    for (int c2 = 0; c2 < kTriB / 2; ++c2) {
                        acc0 = fma(v[c2].x, r[i0 + 2 * c2], acc0);
                        acc1 = fma(v[c2].y, r[i0 + 2 * c2 + 1], acc1);
                    }
                } else {
                    for (int c2 = 0; c2 < n / 2; ++c2) {
                        const double2 v = row[c2];
                        acc0 = fma(v.x, r[i0 + 2 * c2], acc0);
                        acc1 = fma(v.y, r[i0 + 2 * c2 + 1], acc1);
                    }
                }
                r[l] -= acc0 + acc1;
            }
        } else {
            // the rows not yet solved (above the block for UP, else below) less
            // the block's columns times its solution: thread (row q, group g)
            // takes columns 4g .. 4g + 3, so each row's 64 entries are read by 16
            // neighbouring lanes (512 contiguous bytes), and the 16 partial sums
            // are added by butterfly; kTriPass passes of kTriNT / 16 rows each
            // are loaded together
            const int q = tid >> 4, g = tid & 15, c0 = 4 * g;
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = c0 + u < n ? r[i0 + c0 + u] : 0.0;
            for (int l0 = lo; l0 < hi; l0 += kTriPass * (kTriNT / 16)) {
                double acc[kTriPass];
#pragma unroll
                for (int pass = 0; pass < kTriPass; ++pass) {
                    const int l = l0 + pass * (kTriNT / 16) + q;
                    acc[pass] = 0.0;
                    if (l < hi) {
                        const double *row = A + (long long)l * N + i0 + c0;
                        if (c0 + 3 < n) {
                            const double2 v0 = reinterpret_cast<const double2 *>(row)[0];
                            const double2 v1 = reinterpret_cast<const double2 *>(row)[1];
                            acc[pass] = fma(v0.x, x[0], fma(v0.y, x[1], fma(v1.x, x[2], v1.y * x[3])));
                        } else {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (c0 + u < n) acc[pass] = fma(row[u], x[u], acc[pass]);
                        }
                    }
                }
#pragma unroll
                for (int pass = 0; pass < kTriPass; ++pass) {
                    double v = acc[pass];
                    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off);
                    const int l = l0 + pass * (kTriNT / 16) + q;
                    if (g == 0 && l < hi) r[l] -= v;
                }
            }
        }
        __syncthreads();
    }
}

struct TriArgs {
    const AtmDesc *atm;
    const double *A;     // assembled A
    const double *in;
    double *out;
    const int *mask;     // optional per-slab activity mask
    double omega;
    int kind;            // RT_PC_SOR or RT_PC_SSOR
};

// out = P^-1 in.
template <bool ROWWISE>
__global__ __launch_bounds__(kTriNT) void tri_solve_kernel(TriArgs a) {
    extern __shared__ double sm[];
    const int s = blockIdx.x;
    if (a.mask && a.mask[s] == 0) return;
    const AtmDesc at = a.atm[s];
    const int N = 2 * at.ns;
    const double *A = a.A + at.a_off;
    const long long v0 = 2LL * at.doff;
    double *blk = sm;                  // [64][65]
    double *r = sm + kTriB * kTriPad;  // [N]
    for (int i = threadIdx.x; i < N; i += kTriNT) r[i] = a.in[v0 + i];
    __syncthreads();
    tri_sweep<true, false, ROWWISE>(A, N, a.omega, r, blk);
    if (a.kind == RT_PC_SSOR) {
        for (int i = threadIdx.x; i < N; i += kTriNT) r[i] *= A[(long long)i * N + i];
        __syncthreads();
        tri_sweep<false, false, ROWWISE>(A, N, a.omega, r, blk);
        const double sc = (2.0 - a.omega) / a.omega;
        for (int i = threadIdx.x; i < N; i += kTriNT) r[i] *= sc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += kTriNT) a.out[v0 + i] = r[i];
}

// out = P in (the product form, for an initial guess).  One thread per row.
__global__ __launch_bounds__(kTriNT) void tri_mult_kernel(TriArgs a) {
    extern __shared__ double sm[];
    const int s = blockIdx.x;
    const AtmDesc at = a.atm[s];
    const int N = 2 * at.ns;
    const double *A = a.A + at.a_off;
    const long long v0 = 2LL * at.doff;
    const double om = a.omega;
    double *x = sm;
    for (int i = threadIdx.x; i < N; i += kTriNT) x[i] = a.in[v0 + i];
    __syncthreads();
    if (a.kind == RT_PC_SSOR) {
        // t = D^-1 (omega^-1 D + L) x, parked in out (each thread reads back
        // only its own rows), then copied over x once every row has read x
        for (int i = threadIdx.x; i < N; i += kTriNT) {
            const double *row = A + (long long)i * N;
            double acc = row[i] / om * x[i];
            for (int j = 0; j < i; ++j) acc = fma(row[j], x[j], acc);
            a.out[v0 + i] = acc / row[i];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += kTriNT) x[i] = a.out[v0 + i];
        __syncthreads();
    }
    const double sc = a.kind == RT_PC_SSOR ? om / (2.0 - om) : 1.0;
    for (int i = threadIdx.x; i < N; i += kTriNT) {
        const double *row = A + (long long)i * N;
        double acc = row[i] / om * x[i];
        for (int j = i + 1; j < N; ++j) acc = fma(row[j], x[j], acc);
        a.out[v0 + i] = sc * acc;
    }
}

__global__ void fill_kernel(double *v, long long n, double c) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        v[i] = c;
}

// --------------------------------------------------------------------------
// Dense LU with partial pivoting (the direct route of Sect. 3.3 / 4.5: the
// assembled A factored and solved), one workgroup per slab, right-looking in
// panels of NB columns:
//  * the panel's rows live in registers, R rows per thread; each column's
//    pivot is the row of largest magnitude (ties: the lower index), found by
//    a wave butterfly and one LDS pass; the pivot row and the row it replaces
//    are exchanged through LDS, and the pivot row read from there eliminates
//    the column below it -- two barriers per column;
//  * the panel's row exchanges are then applied to the other columns (one
//    thread per column, in order), U12 = L11^-1 A12 is solved one thread per
//    column, and A22 -= L21 U12 streams the trailing rows with the row's
//    L21 in registers and U12 staged in LDS -- within the panel's outer
//    block of BB columns; once the block is factored, the columns beyond it
//    get U12 from the block's BB x BB unit lower triangle and one rank-BB
//    update on the FP64 matrix cores (lu_trailing_mfma).
// piv[k] (slab-local) is the row exchanged with row k at step k, as LAPACK's
// getrf returns it.  A zero pivot marks the slab singular.
// --------------------------------------------------------------------------
constexpr int kLuNT = 512;   // 8 wavefronts; the block's U12 column solve holds BB values
constexpr int kLuNB = 8;     // panel width (16 spills the panel's registers)
constexpr int kLuBB = 32;    // outer block of the few-slab path (multi-workgroup updates)
constexpr int kLuBBBatch = 64;  // the batch kernel's outer block (half the trailing traffic)
constexpr int kLuSplitSlabs = 32;  // batches up to this many slabs: multi-workgroup updates

struct LuArgs {
    const AtmDesc *atm;
    double *LU;    // in: A; out: L (unit, strictly below the diagonal) and U
    int *piv;      // at 2 doff + k
    int *sing;     // per slab: 1 if a pivot was zero
    const int *order;  // workgroup -> slab (largest first), or NULL: workgroup = slab
};

constexpr int kLuUsCols = 128;  // U12 columns staged in LDS per pass of the update
typedef double lu_v4d __attribute__((ext_vector_type(4)));

// A22 -= L21 U12 after outer block K0 (columns K0..K0+BB-1, rows and columns
// from cend on), by the workgroup: U12 is staged in LDS 128 columns at a
// time; each wavefront takes 16-row tiles of the trailing rows, keeps the
// tile's -L21 (16 x BB) as BB / 4 v_mfma_f64_16x16x4 A operands in
// registers, and adds the products to each of the pass's 16 x 16 tiles of
// A22 it loads and stores back.  Each trailing element is read and written
// once per outer block: the batch's factorization is bound by that traffic,
// hence 64-column blocks there.  Operand layout of the instruction: lane l feeds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l is
// D[4 r + l / 16][l % 16].
template <int BB>
__device__ inline void lu_trailing_mfma(double *A, int N, int K0, int cend,
                                        double (*Us)[kLuUsCols]) {
    constexpr int NW = kLuNT / kWave;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int li = lane % 16, lk = lane / 16;
    for (int cc0 = cend; cc0 < N; cc0 += kLuUsCols) {
        __syncthreads();
        for (int e = tid; e < BB * kLuUsCols; e += kLuNT) {
            const int i = e / kLuUsCols, cc = e % kLuUsCols, c = cc0 + cc;
            Us[i][cc] = c < N ? A[(long long)(K0 + i) * N + c] : 0.0;
        }
        __syncthreads();
        for (int r0 = cend + 16 * wave; r0 < N; r0 += 16 * NW) {
            const int ra = r0 + li;
            double av[BB / 4];
#pragma unroll
            for (int kk = 0; kk < BB / 4; ++kk)
                av[kk] = ra < N ? -A[(long long)ra * N + K0 + 4 * kk + lk] : 0.0;
            // the pass's eight 16-column tiles together: their loads in flight
            // at once and eight independent chains of products
            constexpr int CT = kLuUsCols / 16;
            lu_v4d acc[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int col = cc0 + 16 * t + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + 4 * r + lk;
                    acc[t][r] = (row < N && col < N) ? A[(long long)row * N + col] : 0.0;
                }
            }
#pragma unroll
            for (int kk = 0; kk < BB / 4; ++kk)
#pragma unroll
                for (int t = 0; t < CT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], Us[4 * kk + lk][16 * t + li],
                                                                  acc[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int col = cc0 + 16 * t + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + 4 * r + lk;
                    if (row < N && col < N) A[(long long)row * N + col] = acc[t][r];
                }
            }
        }
    }
}

template <int R, int NB, bool SPLIT = false, int BB = kLuBB>
__global__ __launch_bounds__(kLuNT) void lu_factor_kernel(LuArgs g, int K0s = 0) {
    constexpr int NW = kLuNT / kWave;
    __shared__ double swp[2][2][NB];       // [buffer][row j, row p][column]
    __shared__ double redv[2][NW];
    __shared__ int redi[2][NW];
    __shared__ int s_piv[NB];
    __shared__ double L11[NB][NB + 1];
    __shared__ double Lb[BB][BB + 1];   // the outer block's unit lower L11
    extern __shared__ double lu_dyn[];        // U12 columns staged for the update
    double(*Us)[kLuUsCols] = reinterpret_cast<double(*)[kLuUsCols]>(lu_dyn);
    __shared__ double Ub[NB][BB];          // a panel's U12 on the rest of its block
    static_assert(BB % NB == 0, "the outer block is whole panels");
    const int slab = g.order ? g.order[blockIdx.x] : blockIdx.x;
    const AtmDesc at = g.atm[slab];
    const int N = 2 * at.ns;
    double *A = g.LU + at.a_off;
    int *piv = g.piv + 2LL * at.doff;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    int singular = 0;
    // SPLIT: only the outer block at K0s (its swaps and updates confined to
    // the block's columns); the columns outside it are done by the
    // multi-workgroup kernels below
    if (SPLIT && K0s >= N) return;
    if (SPLIT && K0s == 0 && tid == 0) g.sing[slab] = 0;
    for (int k0 = SPLIT ? K0s : 0; k0 < (SPLIT ? min(K0s + BB, N) : N); k0 += NB) {
        const int nb = min(NB, N - k0);
        const int K0 = k0 / BB * BB, cend = min(K0 + BB, N);  // this panel's outer block
        double P[R][NB];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int r = k0 + tid + u * kLuNT;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                P[u][c] = (r < N && c < nb) ? A[(long long)r * N + k0 + c] : 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
            if (jj < nb) {
                const int j = k0 + jj, buf = jj & 1;
                // pivot: largest |P[.][jj]| over rows >= j
                double best = -1.0;
                int bi = N;
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const int r = k0 + tid + u * kLuNT;
                    const double v = fabs(P[u][jj]);
                    if (r >= j && r < N && (v > best || (v == best && r < bi))) {
                        best = v;
                        bi = r;
                    }
                }
                for (int off = kWave / 2; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(best, off);
                    const int oi = __shfl_xor(bi, off);
                    if (ov > best || (ov == best && oi < bi)) {
                        best = ov;
                        bi = oi;
                    }
                }
                if (lane == 0) {
                    redv[buf][wave] = best;
                    redi[buf][wave] = bi;
                }
                __syncthreads();
                best = redv[buf][0];
                bi = redi[buf][0];
                for (int w = 1; w < NW; ++w) {
                    const double ov = redv[buf][w];
                    const int oi = redi[buf][w];
                    if (ov > best || (ov == best && oi < bi)) {
                        best = ov;
                        bi = oi;
                    }
                }
                // no candidate compared (a column of NaNs): keep row j, and
                // the zero test below does not pass a NaN pivot, so mark it
                const int p = bi < N ? bi : j;
                if (bi >= N) singular = 1;
                // exchange rows j and p of the panel through LDS
                const int oj = j - k0, op = p - k0;
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const int lr = tid + u * kLuNT;
                    if (lr == oj)
#pragma unroll
                        for (int c = 0; c < NB; ++c) swp[buf][0][c] = P[u][c];
                    if (lr == op)
#pragma unroll
                        for (int c = 0; c < NB; ++c) swp[buf][1][c] = P[u][c];
                }
                if (tid == 0) s_piv[jj] = p;
                __syncthreads();
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const int lr = tid + u * kLuNT;
                    if (lr == oj)
#pragma unroll
                        for (int c = 0; c < NB; ++c) P[u][c] = swp[buf][1][c];
                    else if (lr == op)
#pragma unroll
                        for (int c = 0; c < NB; ++c) P[u][c] = swp[buf][0][c];
                }
                // eliminate below the pivot (the pivot row is swp[buf][1])
                const double pv = swp[buf][1][jj];
                if (pv == 0.0) singular = 1;
                const double rpv = pv != 0.0 ? 1.0 / pv : 0.0;
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const int r = k0 + tid + u * kLuNT;
                    if (r > j && r < N) {
                        const double l = P[u][jj] * rpv;
                        P[u][jj] = l;
#pragma unroll
                        for (int c = jj + 1; c < NB; ++c) P[u][c] = fma(-l, swp[buf][1][c], P[u][c]);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int r = k0 + tid + u * kLuNT;
            if (r < N)
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < nb) A[(long long)r * N + k0 + c] = P[u][c];
        }
        if (tid < nb) piv[k0 + tid] = s_piv[tid];
        __syncthreads();
        // the panel's row exchanges on the other columns, in order
        for (int c = (SPLIT ? K0 : 0) + tid; c < (SPLIT ? cend : N); c += kLuNT) {
            if (c >= k0 && c < k0 + nb) continue;
            for (int jj = 0; jj < nb; ++jj) {
                const int p = s_piv[jj], j = k0 + jj;
                if (p != j) {
                    const double t = A[(long long)j * N + c];
                    A[(long long)j * N + c] = A[(long long)p * N + c];
                    A[(long long)p * N + c] = t;
                }
            }
        }
        for (int e = tid; e < NB * NB; e += kLuNT) {
            const int r = e / NB, c = e % NB;
            L11[r][c] = (r < nb && c < nb) ? A[(long long)(k0 + r) * N + k0 + c] : 0.0;
        }
        __syncthreads();
        const int c0 = k0 + nb;
        if (c0 >= N) break;
        // U12 = L11^-1 A12 (unit lower L11), one thread per column, on the
        // rest of the outer block (the columns beyond it wait for the block)
        for (int c = c0 + tid; c < cend; c += kLuNT) {
            double u[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) u[i] = i < nb ? A[(long long)(k0 + i) * N + c] : 0.0;
#pragma unroll
            for (int i = 1; i < NB; ++i)
#pragma unroll
                for (int l = 0; l < i; ++l) u[i] = fma(-L11[i][l], u[l], u[i]);
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i < nb) A[(long long)(k0 + i) * N + c] = u[i];
        }
        __syncthreads();
        // A22 -= L21 U12 on the rest of the outer block (at most BB - NB
        // columns): U12 staged in LDS, one thread per trailing row, the row's
        // L21 and block entries loaded together
        __syncthreads();
        for (int e = tid; e < NB * BB; e += kLuNT) {
            const int i = e / BB, cc = e % BB, c = c0 + cc;
            Ub[i][cc] = (i < nb && c < cend) ? A[(long long)(k0 + i) * N + c] : 0.0;
        }
        __syncthreads();
        for (int r = c0 + tid; r < N; r += kLuNT) {
            // a compiler-only barrier: Ub is read from LDS per row rather than
            // kept in registers across the loop
            asm volatile("" ::: "memory");
            double l[NB], v[BB - NB];
            const double *row = A + (long long)r * N;
#pragma unroll
            for (int i = 0; i < NB; ++i) l[i] = i < nb ? row[k0 + i] : 0.0;
#pragma unroll
            for (int cc = 0; cc < BB - NB; ++cc) v[cc] = c0 + cc < cend ? row[c0 + cc] : 0.0;
#pragma unroll
            for (int cc = 0; cc < BB - NB; ++cc) {
#pragma unroll
                for (int i = 0; i < NB; ++i) v[cc] = fma(-l[i], Ub[i][cc], v[cc]);
                if (c0 + cc < cend) A[(long long)r * N + c0 + cc] = v[cc];
            }
        }
        __syncthreads();
        if (SPLIT || c0 < cend || cend >= N) continue;
        // the outer block is factored: U12 = Lb^-1 A12 on the columns beyond
        // it (one thread per column, written back), then A22 -= L21 U12 for
        // the trailing rows and columns on the FP64 matrix cores
        for (int e = tid; e < BB * BB; e += kLuNT) {
            const int r = e / BB, c = e % BB;
            Lb[r][c] = A[(long long)(K0 + r) * N + K0 + c];
        }
        __syncthreads();
        for (int c = cend + tid; c < N; c += kLuNT) {
            // a compiler-only barrier: Lb is read from LDS per column rather
            // than hoisted into registers (496 of them) across the loop
            asm volatile("" ::: "memory");
            double u[BB];
#pragma unroll
            for (int i = 0; i < BB; ++i) u[i] = A[(long long)(K0 + i) * N + c];
#pragma unroll
            for (int i = 1; i < BB; ++i)
#pragma unroll
                for (int l = 0; l < i; ++l) u[i] = fma(-Lb[i][l], u[l], u[i]);
#pragma unroll
            for (int i = 0; i < BB; ++i) A[(long long)(K0 + i) * N + c] = u[i];
        }
        lu_trailing_mfma<BB>(A, N, K0, cend, Us);
        __syncthreads();
    }
    if (tid == 0) {
        if (!SPLIT) g.sing[slab] = singular;
        else if (singular) g.sing[slab] = 1;
    }
}

// Multi-workgroup completion of outer block K0 (few large slabs), after
// lu_factor_kernel<..., true> has factored the block's columns:
//  * lu_swap_u12_kernel, one wavefront per (slab, 64-column tile): the
//    block's row exchanges, in order, on every column outside the block, then
//    U12 = Lb^-1 A12 for the tile's columns right of the block;
//  * lu_rank32_kernel, one workgroup per (slab, 64-column tile, 128-row
//    tile): A22 -= L21 U12 with U12 and L21 staged in LDS.
constexpr int kLuTileC = 64, kLuTileR = 128;

__global__ __launch_bounds__(kWave) void lu_swap_u12_kernel(LuArgs g, int K0) {
    __shared__ double Lb[kLuBB][kLuBB + 1];
    __shared__ int sp[kLuBB];
    const int slab = blockIdx.y;
    const AtmDesc at = g.atm[slab];
    const int N = 2 * at.ns;
    if (K0 >= N) return;
    const int t0 = blockIdx.x * kLuTileC;
    if (t0 >= N) return;
    double *A = g.LU + at.a_off;
    const int *piv = g.piv + 2LL * at.doff;
    const int cend = min(K0 + kLuBB, N), nbk = cend - K0, tid = threadIdx.x;
    if (tid < nbk) sp[tid] = piv[K0 + tid];
    for (int e = tid; e < kLuBB * kLuBB; e += kWave) {
        const int r = e / kLuBB, c = e % kLuBB;
        Lb[r][c] = (r < nbk && c < nbk) ? A[(long long)(K0 + r) * N + K0 + c] : 0.0;
    }
    __syncthreads();
    const int c = t0 + tid;
    if (c >= N || (c >= K0 && c < cend)) return;
    for (int i = 0; i < nbk; ++i) {
        const int p = sp[i], j = K0 + i;
        if (p != j) {
            const double t = A[(long long)j * N + c];
            A[(long long)j * N + c] = A[(long long)p * N + c];
            A[(long long)p * N + c] = t;
        }
    }
    if (c < cend) return;  // left of the block: the exchanges only
    // right of the block: there are such columns only when the block is
    // whole (nbk = kLuBB), so no row guards
    double u[kLuBB];
#pragma unroll
    for (int i = 0; i < kLuBB; ++i) u[i] = A[(long long)(K0 + i) * N + c];
#pragma unroll
    for (int i = 1; i < kLuBB; ++i)
#pragma unroll
        for (int l = 0; l < i; ++l) u[i] = fma(-Lb[i][l], u[l], u[i]);
#pragma unroll
    for (int i = 0; i < kLuBB; ++i) A[(long long)(K0 + i) * N + c] = u[i];
}

__global__ __launch_bounds__(256) void lu_rank32_kernel(LuArgs g, int K0) {
    __shared__ double U[kLuBB][kLuTileC];
    __shared__ double L[kLuTileR][kLuBB + 1];
    const int slab = blockIdx.z;
    const AtmDesc at = g.atm[slab];
    const int N = 2 * at.ns, cend = K0 + kLuBB;
    if (cend >= N) return;  // no trailing matrix (or the last, partial block)
    const int t0 = cend + blockIdx.x * kLuTileC, r0 = cend + blockIdx.y * kLuTileR;
    if (t0 >= N || r0 >= N) return;
    double *A = g.LU + at.a_off;
    const int tid = threadIdx.x, cl = tid % kLuTileC, rg = tid / kLuTileC;  // 4 row lanes
    for (int e = tid; e < kLuBB * kLuTileC; e += 256) {
        const int i = e / kLuTileC, cc = e % kLuTileC;
        U[i][cc] = t0 + cc < N ? A[(long long)(K0 + i) * N + t0 + cc] : 0.0;
    }
    const int nr = min(kLuTileR, N - r0);
    for (int e = tid; e < kLuTileR * kLuBB; e += 256) {
        const int rr = e / kLuBB, i = e % kLuBB;
        L[rr][i] = rr < nr ? A[(long long)(r0 + rr) * N + K0 + i] : 0.0;
    }
    __syncthreads();
    const int c = t0 + cl;
    if (c >= N) return;
    double u[kLuBB];
#pragma unroll
    for (int i = 0; i < kLuBB; ++i) u[i] = U[i][cl];
    // rows rg, rg + 4, ...: 16 of them loaded together, twice
    for (int h = 0; h < kLuTileR / 4; h += 16) {
        double a[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int rr = rg + 4 * (h + t);
            a[t] = rr < nr ? A[(long long)(r0 + rr) * N + c] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int rr = rg + 4 * (h + t);
#pragma unroll
            for (int i = 0; i < kLuBB; ++i) a[t] = fma(-L[rr][i], u[i], a[t]);
            if (rr < nr) A[(long long)(r0 + rr) * N + c] = a[t];
        }
    }
}

// x = A^-1 b from the factors: row exchanges, L y = P b, U x = y.
template <bool ROWWISE>
__global__ __launch_bounds__(kTriNT) void lu_solve_kernel(const AtmDesc *atm, const double *LU,
                                                          const int *pivs, const double *b,
                                                          double *x) {
    extern __shared__ double sm[];
    const int s = blockIdx.x;
    const AtmDesc at = atm[s];
    const int N = 2 * at.ns;
    const double *A = LU + at.a_off;
    const int *piv = pivs + 2LL * at.doff;
    const long long v0 = 2LL * at.doff;
    double *blk = sm;
    double *r = sm + kTriB * kTriPad;
    for (int i = threadIdx.x; i < N; i += kTriNT) r[i] = b[v0 + i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < N; ++k) {
            const int p = piv[k];
            if (p != k) {
                const double t = r[k];
                r[k] = r[p];
                r[p] = t;
            }
        }
    __syncthreads();
    tri_sweep<false, true, ROWWISE>(A, N, 1.0, r, blk);
    tri_sweep<true, false, ROWWISE>(A, N, 1.0, r, blk);
    for (int i = threadIdx.x; i < N; i += kTriNT) x[v0 + i] = r[i];
}

size_t tri_lds(int ns_max) { return (size_t)(kTriB * kTriPad + 2 * ns_max) * sizeof(double); }

template <typename K>
hipError_t lds_limit(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

TriArgs tri_args(const rt_handle *h, const double *in, double *out, const int *mask) {
    TriArgs a{};
    a.atm = h->d_atm;
    a.A = h->d_A;
    a.in = in;
    a.out = out;
    a.mask = mask;
    a.omega = h->opt.omega;
    a.kind = h->opt.precond;
    return a;
}

// Few slabs (fewer workgroups than CUs): each workgroup's own loads in flight
// decide its speed, so one thread per row with the row's 64 entries loaded
// together; many slabs: the coalesced 16-lanes-per-row update.
bool tri_rowwise(const rt_handle *h) { return h->n_atm < 256; }

}  // namespace

hipError_t precond_tri(const rt_handle *h, const double *in, double *out, const int *mask,
                       hipStream_t s) {
    const size_t lds = tri_lds(h->ns_max);
    const TriArgs a = tri_args(h, in, out, mask);
    if (tri_rowwise(h)) {
        hipError_t e = lds_limit(tri_solve_kernel<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(tri_solve_kernel<true>, dim3(h->n_atm), dim3(kTriNT), lds, s, a);
    } else {
        hipError_t e = lds_limit(tri_solve_kernel<false>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(tri_solve_kernel<false>, dim3(h->n_atm), dim3(kTriNT), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t precond_tri_mult(const rt_handle *h, const double *in, double *out, hipStream_t s) {
    const size_t lds = (size_t)2 * h->ns_max * sizeof(double);
    hipError_t e = lds_limit(tri_mult_kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tri_mult_kernel, dim3(h->n_atm), dim3(kTriNT), lds, s,
                       tri_args(h, in, out, nullptr));
    return hipGetLastError();
}

hipError_t fill(double *v, long long n, double c, hipStream_t s) {
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, v, n, c);
    return hipGetLastError();
}

int lu_factor(rt_handle *h, hipStream_t s) {
    if (h->lu_ready) return RT_OK;
    if (h->fs == RT_FS_DELO_PARABOLIC)
        return fail(RT_EINVAL, "the LU route supports the two-point formal solvers only");
    const size_t bytes = sizeof(double) * (size_t)std::max<long long>(h->n_dense, 1);
    if (!h->d_LU) {
        // all four or none: a failed allocation frees the others, so a later
        // call starts over instead of finding a partial set
        if (hipMalloc((void **)&h->d_LU, bytes) != hipSuccess ||
            hipMalloc((void **)&h->d_piv, sizeof(int) * h->n_unk) != hipSuccess ||
            hipMalloc((void **)&h->d_sing, sizeof(int) * h->n_atm) != hipSuccess ||
            hipMalloc((void **)&h->d_lu_order, sizeof(int) * h->n_atm) != hipSuccess) {
            (void)hipGetLastError();
            for (void **p : {(void **)&h->d_LU, (void **)&h->d_piv, (void **)&h->d_sing,
                             (void **)&h->d_lu_order}) {
                if (*p) (void)hipFree(*p);
                *p = nullptr;
            }
            return fail(RT_ENOMEM, "device allocation of the LU factors failed");
        }
        // one workgroup per slab, dispatched in order: the largest slabs first,
        // so that the small ones fill in behind them (a factorization costs
        // about N^3)
        std::vector<int> order(h->n_atm);
        for (int i = 0; i < h->n_atm; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return h->ns[x] > h->ns[y]; });
        if (hipMemcpy(h->d_lu_order, order.data(), sizeof(int) * h->n_atm,
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RT_EDEVICE, "copy of the factorization order failed");
        }
    }
    int rc = h->dense_ready ? RT_OK : assemble(h, h->d_LU, s);
    if (rc != RT_OK) return rc;
    if (h->dense_ready &&
        hipMemcpyAsync(h->d_LU, h->d_A, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(RT_EDEVICE, "copy of the assembled operator failed");
    LuArgs g{h->d_atm, h->d_LU, h->d_piv, h->d_sing, nullptr};
    const int N = 2 * h->ns_max;
    if (h->n_atm <= kLuSplitSlabs && N > kLuBB) {
        // few slabs: each 32-column block factored by one workgroup per slab,
        // the rest of the matrix updated by workgroups over column and row tiles
        for (int K0 = 0; K0 < N; K0 += kLuBB) {
            if (N <= kLuNT)
                hipLaunchKernelGGL((lu_factor_kernel<1, kLuNB, true>), dim3(h->n_atm), dim3(kLuNT), 0, s, g, K0);
            else if (N <= 2 * kLuNT)
                hipLaunchKernelGGL((lu_factor_kernel<2, kLuNB, true>), dim3(h->n_atm), dim3(kLuNT), 0, s, g, K0);
            else if (N <= 4 * kLuNT)
                hipLaunchKernelGGL((lu_factor_kernel<4, kLuNB, true>), dim3(h->n_atm), dim3(kLuNT), 0, s, g, K0);
            else
                hipLaunchKernelGGL((lu_factor_kernel<8, kLuNB, true>), dim3(h->n_atm), dim3(kLuNT), 0, s, g, K0);
            hipLaunchKernelGGL(lu_swap_u12_kernel, dim3((N + kLuTileC - 1) / kLuTileC, h->n_atm),
                               dim3(kWave), 0, s, g, K0);
            const int rest = N - K0 - kLuBB;
            if (rest > 0)
                hipLaunchKernelGGL(lu_rank32_kernel,
                                   dim3((rest + kLuTileC - 1) / kLuTileC, (rest + kLuTileR - 1) / kLuTileR, h->n_atm),
                                   dim3(256), 0, s, g, K0);
            if (hipGetLastError() != hipSuccess) return fail(RT_EDEVICE, "LU factorization launch failed");
        }
        h->lu_ready = true;
        return RT_OK;
    }
    g.order = h->d_lu_order;
    // one workgroup per slab with 64-column outer blocks; their U12 stage
    // (64 x kLuUsCols doubles) in dynamic LDS
    const size_t lds = (size_t)kLuBBBatch * kLuUsCols * sizeof(double);
    auto launch = [&](auto kernel) {
        if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return;  // the launch below reports the error
        hipLaunchKernelGGL(kernel, dim3(h->n_atm), dim3(kLuNT), lds, s, g, 0);
    };
    if (N <= kLuNT)
        launch(lu_factor_kernel<1, kLuNB, false, kLuBBBatch>);
    else if (N <= 2 * kLuNT)
        launch(lu_factor_kernel<2, kLuNB, false, kLuBBBatch>);
    else if (N <= 4 * kLuNT)
        launch(lu_factor_kernel<4, kLuNB, false, kLuBBBatch>);
    else
        launch(lu_factor_kernel<8, kLuNB, false, kLuBBBatch>);
    if (hipGetLastError() != hipSuccess) return fail(RT_EDEVICE, "LU factorization launch failed");
    h->lu_ready = true;
    return RT_OK;
}

hipError_t lu_solve(const rt_handle *h, const double *b, double *x, hipStream_t s) {
    const size_t lds = tri_lds(h->ns_max);
    const AtmDesc *atm = h->d_atm;
    const double *LU = h->d_LU;
    const int *piv = h->d_piv;
    if (tri_rowwise(h)) {
        hipError_t e = lds_limit(lu_solve_kernel<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(lu_solve_kernel<true>, dim3(h->n_atm), dim3(kTriNT), lds, s, atm, LU, piv,
                           b, x);
    } else {
        hipError_t e = lds_limit(lu_solve_kernel<false>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(lu_solve_kernel<false>, dim3(h->n_atm), dim3(kTriNT), lds, s, atm, LU,
                           piv, b, x);
    }
    return hipGetLastError();
}

int ensure_dense(rt_handle *h, hipStream_t s) {
    if (h->dense_ready) return RT_OK;
    if (h->fs == RT_FS_DELO_PARABOLIC)
        return fail(RT_EINVAL, "SOR and SSOR support the two-point formal solvers only");
    if (!h->d_A) {
        if (hipMalloc((void **)&h->d_A, sizeof(double) * (size_t)std::max<long long>(h->n_dense, 1)) !=
            hipSuccess) {
            h->d_A = nullptr;
            (void)hipGetLastError();
            return fail(RT_ENOMEM, "device allocation of the assembled operator failed");
        }
    }
    const int rc = assemble(h, h->d_A, s);
    if (rc != RT_OK) return rc;
    h->dense_ready = true;
    return RT_OK;
}

}  // namespace rt
