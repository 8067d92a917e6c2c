// Structured multipliers applied by FFT.
//
// A circulant C = (c_{(i-j) mod n}) is diagonalised by the DFT (Theorem thcpw),
// so a product with C costs O(n log n) per vector instead of O(n^2) (Section 6:
// the product A C takes order n^2 log n flops against 2n^3 - n^2 for a dense
// multiplier).  A Toeplitz matrix T = (t_{i-j}) is the leading block of a
// circulant of any period m >= 2n - 1, and is applied the same way after zero
// padding.  With h the period-m first column (h[d mod m] = t_d):
//   row of A H   : y_j = sum_k a_k h[(k - j) mod m]   (correlation: X conj(H))
//   H y          : y_j = sum_k h[(j - k) mod m] y_k  (convolution: X H)
//   H^T w        : correlation again.
//
// One workgroup transforms one vector.  The real length-m signal is packed as
// z_k = x_{2k} + i x_{2k+1} (k < L = m/2) and transformed by a complex FFT of
// length L in radix-16 Stockham passes (registers, with LDS between passes);
// the real spectrum is untangled pairwise (f, L - f), multiplied by the
// kernel's spectrum, re-packed, and sent back through the inverse passes,
// whose last one writes the row.  Twiddles e^{-i pi j / L}, j = 0..L, come
// from a table built once per multiplier.
//
// Bound: HBM for the row transform (one read and one write of each element)
// when LDS and VALU keep up; 5 m log2 m flops per vector (forward + inverse).
#include "rmge_impl.h"

namespace rmge {
namespace {

struct cplx {
    double x, y;
};
__device__ inline cplx operator+(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline cplx operator-(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline cplx cmul(cplx a, cplx b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ inline cplx cconj(cplx a) { return {a.x, -a.y}; }
__device__ inline cplx cscale(cplx a, double s) { return {a.x * s, a.y * s}; }


__global__ void k_twiddles(int L, cplx *tw) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j <= L; j += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-static_cast<double>(j) / static_cast<double>(L), &s, &c);
        tw[j] = {c, s};
    }
}

// ---------------------------------------------------------------------------
// Row transforms as Stockham passes (Govindaraju et al., SC'08 formulation of
// the autosorting FFT): a complex length L = 2^LOGL is done in passes of
// radix 16 (the last one 2, 4 or 8 when LOGL is not a multiple of 4).  Each of
// the T = L / 16 threads of a workgroup holds 16 values in registers; in a
// pass of radix R it takes the butterflies j = tid + q T (q < 16 / R):
//   inputs    a_r = z[j + r L / R]                 (consecutive j: coalesced)
//   twiddles  a_r *= w^{r k},  k = j mod Ns,  w = e^{-2 pi i / (Ns R)}
//   DFT_R     b_s = sum_r a_r e^{-2 pi i r s / R}  (in registers)
//   outputs   z[(j / Ns) Ns R + k + s Ns] = b_s    (Ns = product of the
//                                                    earlier passes' radices)
// and the result comes out in natural order.  Values move between passes
// through LDS (one complex of padding per 16, against bank conflicts); the
// first forward pass reads the row straight from global memory and the last
// inverse pass writes it straight back, both as whole 16-byte (or 8-byte)
// elements z_k = (x_{2k}, x_{2k+1}) across consecutive lanes.  Pass twiddles
// come from the table e^{-i pi t / L}, t = 0..L, by symmetry beyond t = L.

// x e^{-2 pi i a / 16} (forward) or x e^{+2 pi i a / 16} (inverse), a a
// compile-time constant after unrolling.
__device__ inline cplx rot16(cplx x, int a, bool inv) {
    constexpr double C1 = 0.92387953251128675613;  // cos(pi / 8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi / 8)
    constexpr double R2 = 0.70710678118654752440;  // sqrt(2) / 2
    a &= 15;
    if (a == 0) return x;
    // e^{-2 pi i a / 16} = c + i s
    double c, sn;
    switch (a & 7) {
    case 0: c = 1.0; sn = 0.0; break;
    case 1: c = C1; sn = -S1; break;
    case 2: c = R2; sn = -R2; break;
    case 3: c = S1; sn = -C1; break;
    case 4: c = 0.0; sn = -1.0; break;
    case 5: c = -S1; sn = -C1; break;
    case 6: c = -R2; sn = -R2; break;
    default: c = -C1; sn = -S1; break;
    }
    if (a & 8) { c = -c; sn = -sn; }
    if (inv) sn = -sn;
    if ((a & 3) == 0) {  // multiples of -pi/2: exact swaps and sign changes
        if (a == 8) return {-x.x, -x.y};
        return sn < 0 ? cplx{x.y, -x.x} : cplx{-x.y, x.x};
    }
    return {x.x * c - x.y * sn, x.x * sn + x.y * c};
}

__device__ inline int brev_c(int r, int bits) {
    int o = 0;
    for (int b = 0; b < bits; ++b) o |= ((r >> b) & 1) << (bits - 1 - b);
    return o;
}

// b_s = sum_r a_r e^{-+2 pi i r s / R} in place, R in {2, 4, 8, 16}.
template <int R>
__device__ inline void dft_reg(cplx *a, bool inv) {
    constexpr int BITS = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    cplx b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[brev_c(r, BITS)] = a[r];
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const cplx u = b[g + k];
                const cplx v = rot16(b[g + k + h], k * (8 / h), inv);
                b[g + k] = u + v;
                b[g + k + h] = u - v;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = b[r];
}

__device__ inline int lds_pad(int i) { return i + (i >> 4); }

// A complex value to or from LDS as one 16-byte access (ds_read_b128 /
// ds_write_b128): as two 8-byte halves, consecutive lanes' accesses 16 bytes
// apart fall on every other bank pair and conflict two ways.
__device__ inline cplx lds_get(const cplx *sm, int i) {
    const double2 v = reinterpret_cast<const double2 *>(sm)[i];
    return {v.x, v.y};
}
__device__ inline void lds_put(cplx *sm, int i, cplx v) {
    reinterpret_cast<double2 *>(sm)[i] = double2{v.x, v.y};
}

// Radix of pass p (0-based) of a length-2^LOGL transform: 16 while four bits
// remain, then the rest.
template <int LOGL>
struct Passes {
    static constexpr int kFull = LOGL / 4, kRest = LOGL % 4;
    static constexpr int kCount = kFull + (kRest ? 1 : 0);
    __host__ __device__ static constexpr int radix(int p) { return p < kFull ? 16 : 1 << kRest; }
    __host__ __device__ static constexpr int ns(int p) {  // product of the earlier radices
        return p == 0 ? 1 : ns(p - 1) * radix(p - 1);
    }
};

// e^{-i pi t / L} for 0 <= t < 2 L from the table of t <= L (the rest by symmetry).
__device__ inline cplx tw_at(const cplx *__restrict__ tw, int t, int L) {
    const cplx w = tw[t <= L ? t : t - L];
    return t <= L ? w : cplx{-w.x, -w.y};
}

// Twiddles and DFT of pass P on the thread's registers a[16] (inputs as
// gathered by the pass), leaving the pass outputs in a.
template <int LOGL, int P>
__device__ inline void pass_compute(cplx *a, int tid, const cplx *__restrict__ tw, bool inv) {
    constexpr int L = 1 << LOGL, R = Passes<LOGL>::radix(P), NS = Passes<LOGL>::ns(P);
    constexpr int T = L >= 16 ? L / 16 : 1, Q = (L >= 16 ? 16 : L) / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = tid + q * T;
        if (NS > 1) {
            // w^{r k} = e^{-i pi r t / L}, t = 2 k L / (NS R): each power from the
            // table (correctly rounded; products of powers would add roundings)
            const int k = j & (NS - 1), t = 2 * k * (L / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx w = tw_at(tw, r * t, L);
                a[q * R + r] = cmul(a[q * R + r], inv ? cconj(w) : w);
            }
        }
        dft_reg<R>(a + q * R, inv);
    }
}

// Store pass P's outputs into LDS, natural Stockham order.
template <int LOGL, int P>
__device__ inline void pass_store(const cplx *a, int tid, cplx *sm) {
    constexpr int L = 1 << LOGL, R = Passes<LOGL>::radix(P), NS = Passes<LOGL>::ns(P);
    constexpr int T = L >= 16 ? L / 16 : 1, Q = (L >= 16 ? 16 : L) / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = tid + q * T, k = j & (NS - 1), base = (j / NS) * NS * R + k;
#pragma unroll
        for (int s = 0; s < R; ++s) lds_put(sm, lds_pad(base + s * NS), a[q * R + s]);
    }
}

// Gather pass P's inputs from LDS.
template <int LOGL, int P>
__device__ inline void pass_load(cplx *a, int tid, const cplx *sm) {
    constexpr int L = 1 << LOGL, R = Passes<LOGL>::radix(P);
    constexpr int T = L >= 16 ? L / 16 : 1, Q = (L >= 16 ? 16 : L) / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = tid + q * T;
#pragma unroll
        for (int r = 0; r < R; ++r) a[q * R + r] = lds_get(sm, lds_pad(j + r * (L / R)));
    }
}

// Passes P .. end of one transform: compute pass P on a, then for every later
// pass store, barrier, load, compute.  On return a holds the last pass's
// outputs (not stored).
template <int LOGL, int P>
__device__ inline void run_passes(cplx *a, int tid, bool active, cplx *sm,
                                  const cplx *__restrict__ tw, bool inv) {
    if constexpr (P < Passes<LOGL>::kCount) {
        if (active) pass_compute<LOGL, P>(a, tid, tw, inv);
        if constexpr (P + 1 < Passes<LOGL>::kCount) {
            if (active) pass_store<LOGL, P>(a, tid, sm);
            __syncthreads();
            if (active) pass_load<LOGL, P + 1>(a, tid, sm);
            __syncthreads();
            run_passes<LOGL, P + 1>(a, tid, active, sm, tw, inv);
        }
    }
}

// z_e = (x_{2e}, x_{2e+1}) of a row zero padded beyond n.  The loads are issued
// unconditionally (from a clamped, in-range address, the value then selected),
// so a whole gather is in flight at once: a load under a branch would be
// waited for where the branch rejoins.
template <typename TI>
__device__ inline cplx load_pair(const TI *x, int64_t esi, int64_t n, int64_t e) {
    const int64_t j0 = 2 * e, j1 = j0 + 1;
    if (esi == 1 && (n & 1) == 0) {  // whole pairs: one 16-byte (8-byte) load
        const bool in = j0 < n;
        const TI *p = x + (in ? j0 : 0);
        if constexpr (sizeof(TI) == 8) {
            const double2 v = *reinterpret_cast<const double2 *>(p);
            return in ? cplx{v.x, v.y} : cplx{0.0, 0.0};
        } else {
            const float2 v = *reinterpret_cast<const float2 *>(p);
            return in ? cplx{static_cast<double>(v.x), static_cast<double>(v.y)} : cplx{0.0, 0.0};
        }
    }
    const double re = static_cast<double>(load_if(x, j0 * esi, j0 < n));
    const double im = static_cast<double>(load_if(x, j1 * esi, j1 < n));
    return {re, im};
}

// One row x (n values, element stride esi, zero padded to the period m):
//   spec != null: the half spectrum X_0 .. X_L of x into spec;
//   else y = beta y + (x correlated (conj = 1) / convolved (conj = 0) with the
//   period-m kernel of half spectrum hhat), the first n values, stride eso,
// with the transforms done as Stockham passes; LOGL = log2(m / 2), m >= 2.
// Called by every thread of a workgroup of at least max(64, L / 16) threads
// (the barriers are workgroup-wide); sm: (L + L / 16 + 1) complex of LDS.
// The first forward pass's inputs z_e, e = j + r L / R, gathered from the row.
template <int LOGL, typename TI>
__device__ inline void fft_gather(cplx *a, const TI *x, int64_t esi, int64_t n) {
    constexpr int L = 1 << LOGL;
    constexpr int T = L >= 16 ? L / 16 : 1, V = L >= 16 ? 16 : L;
    constexpr int P0R = Passes<LOGL>::kCount ? Passes<LOGL>::radix(0) : 1;
    const int tid = threadIdx.x;
    if (tid >= T) return;
#pragma unroll
    for (int q = 0; q < V / P0R; ++q)
#pragma unroll
        for (int r = 0; r < P0R; ++r)
            a[q * P0R + r] = load_pair(x, esi, n, tid + q * T + r * (L / P0R));
}

// The rest of the row operation, from the gathered inputs in a.
template <int LOGL, typename TO>
__device__ inline void fft_row_regs(cplx *a, int64_t n, const cplx *__restrict__ tw,
                                    const cplx *__restrict__ hhat, int conj, double beta, TO *y,
                                    int64_t eso, cplx *spec, double *absmax, cplx *sm) {
    constexpr int L = 1 << LOGL;
    constexpr int T = L >= 16 ? L / 16 : 1;   // threads holding data
    constexpr int V = L >= 16 ? 16 : L;       // values per thread
    const int tid = threadIdx.x;
    const bool active = tid < T;
    run_passes<LOGL, 0>(a, tid, active, sm, tw, false);
    // spectrum Z_f in natural order, f = j + s L / R of the last pass
    if (active) {
        constexpr int PL = Passes<LOGL>::kCount ? Passes<LOGL>::kCount - 1 : 0;
        constexpr int RL = Passes<LOGL>::kCount ? Passes<LOGL>::radix(PL) : 1;
#pragma unroll
        for (int q = 0; q < V / RL; ++q)
#pragma unroll
            for (int s2 = 0; s2 < RL; ++s2)
                lds_put(sm, lds_pad(tid + q * T + s2 * (L / RL)), a[q * RL + s2]);
    }
    __syncthreads();
    // pairs (f, L - f): untangle the real spectrum, apply the kernel, re-pack
    // (the workgroup has BD = max(64, L / 16) threads)
    constexpr int BD = L / 16 > 64 ? L / 16 : 64;
#pragma unroll 1
    for (int qf = 0; qf < (L / 2 + BD) / BD; ++qf) {
        const int f = tid + qf * BD;
        if (f > L / 2) break;
        const int g = (L - f) & (L - 1);
        const cplx Zf = lds_get(sm, lds_pad(f)), Zg = lds_get(sm, lds_pad(g));
        const cplx e = cscale(Zf + cconj(Zg), 0.5);
        const cplx dd = Zf - cconj(Zg);
        const cplx o = {0.5 * dd.y, -0.5 * dd.x};  // -i/2 (Z_f - conj Z_{L-f})
        const cplx w = tw[f];                       // e^{-2 pi i f / m}
        const cplx wo = cmul(w, o);
        const cplx Xf = e + wo;                     // X_f
        const cplx Xg = cconj(e - wo);              // X_{L-f} (X_L when f = 0)
        if (spec != nullptr) {
            spec[f] = Xf;
            if (f == 0)
                spec[L] = Xg;
            else if (g != f)
                spec[g] = Xg;
            continue;
        }
        cplx Hf = hhat[f], Hg = hhat[L - f];
        if (conj) {
            Hf = cconj(Hf);
            Hg = cconj(Hg);
        }
        const cplx Yf = cmul(Xf, Hf), Yg = cmul(Xg, Hg);
        const cplx ep = cscale(Yf + cconj(Yg), 0.5);
        const cplx op = cscale(cmul(Yf - cconj(Yg), cconj(w)), 0.5);
        lds_put(sm, lds_pad(f), {ep.x - op.y, ep.y + op.x});  // E' + i O'
        if (f != 0 && g != f) {
            const cplx ec = cconj(ep), oc = cconj(op);
            lds_put(sm, lds_pad(g), {ec.x - oc.y, ec.y + oc.x});
        }
    }
    if (spec != nullptr) return;
    __syncthreads();
    // inverse transform: gather the first pass's inputs from LDS, run, and
    // write the last pass's outputs (natural order e = j + s L / R) to the row
    if (active) pass_load<LOGL, 0>(a, tid, sm);
    __syncthreads();  // every input read before the first pass stores over them
    run_passes<LOGL, 0>(a, tid, active, sm, tw, true);
    const double scale = 1.0 / static_cast<double>(L);
    double vmax = 0.0;  // stays 0 in the threads that hold no data
    constexpr int PL = Passes<LOGL>::kCount ? Passes<LOGL>::kCount - 1 : 0;
    constexpr int RL = Passes<LOGL>::kCount ? Passes<LOGL>::radix(PL) : 1;
#pragma unroll
    for (int q = 0; q < (active ? V / RL : 0); ++q)
#pragma unroll
        for (int s2 = 0; s2 < RL; ++s2) {
            const int64_t e = tid + q * T + s2 * (L / RL);
            const cplx zz = a[q * RL + s2];
            const int64_t j0 = 2 * e, j1 = j0 + 1;
            double v0 = zz.x * scale, v1 = zz.y * scale;
            if (eso == 1 && j1 < n) {
                TO *p = y + j0;
                if (beta != 0.0) {
                    v0 += beta * static_cast<double>(p[0]);
                    v1 += beta * static_cast<double>(p[1]);
                }
                if constexpr (sizeof(TO) == 8) {
                    *reinterpret_cast<double2 *>(p) = double2{v0, v1};
                } else {
                    *reinterpret_cast<float2 *>(p) =
                        float2{static_cast<float>(v0), static_cast<float>(v1)};
                }
                vmax = fmax(vmax, fmax(fabs(static_cast<double>(static_cast<TO>(v0))),
                                       fabs(static_cast<double>(static_cast<TO>(v1)))));
                continue;
            }
            if (j0 < n) {
                TO *p = y + j0 * eso;
                const TO o = static_cast<TO>(beta == 0.0 ? v0 : beta * static_cast<double>(*p) + v0);
                *p = o;
                vmax = fmax(vmax, fabs(static_cast<double>(o)));
            }
            if (j1 < n) {
                TO *p = y + j1 * eso;
                const TO o = static_cast<TO>(beta == 0.0 ? v1 : beta * static_cast<double>(*p) + v1);
                *p = o;
                vmax = fmax(vmax, fabs(static_cast<double>(o)));
            }
        }
    if (absmax != nullptr) {  // max |out| for the growth statistic, one atomic per wave
        for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
        if ((tid & 63) == 0)
            atomicMax(reinterpret_cast<unsigned long long *>(absmax),
                      static_cast<unsigned long long>(__double_as_longlong(vmax)));
    }
}

template <int LOGL, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline void fft_row(const TI *x, int64_t esi, int64_t n, const cplx *__restrict__ tw,
                               const cplx *__restrict__ hhat, int conj, double beta, TO *y,
                               int64_t eso, cplx *spec, double *absmax, cplx *sm) {
    cplx a[16];
    fft_gather<LOGL, TI>(a, x, esi, n);
    fft_row_regs<LOGL, TO>(a, n, tw, hhat, conj, beta, y, eso, spec, absmax, sm);
}

// One row a workgroup: row v of `in` (stride vsi) to row v of `out` (stride vso).
template <int LOGL, typename TI, typename TO>
__global__ __launch_bounds__((1 << LOGL) >= 1024 ? (1 << LOGL) / 16 : 64) void k_fft_stockham(
    const TI *in, int64_t vsi, int64_t esi, int64_t n, const cplx *__restrict__ tw,
    const cplx *__restrict__ hhat, int conj, double beta, TO *out, int64_t vso, int64_t eso,
    cplx *spec, double *absmax) {
    extern __shared__ cplx sm[];
    const int64_t v = blockIdx.x;
    fft_row<LOGL, TI, TO>(in + v * vsi, esi, n, tw, hhat, conj, beta, out + v * vso, eso, spec,
                          absmax, sm);
}

// Period-m kernel h from the multiplier parameters:
//   circulant, m == n   : h[d] = c[d]
//   circulant, m >= 2n-1: h[d] = c[d], h[m-d] = c[n-d] (d = 1..n-1)  (t_d = c[d mod n])
//   Toeplitz,  m >= 2n-1: h[d] = tau[d], h[m-d] = tau[n-1+d] (d = 1..n-1)
__global__ void k_embed(int kind, const double *p, int64_t n, int m, double *h) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (kind == 2 && m == n) {
            v = p[j];
        } else if (j < n) {
            v = p[j];
        } else if (j > m - n) {
            const int64_t d = m - j;  // 1..n-1
            v = (kind == 2) ? p[n - d] : p[n - 1 + d];
        }
        h[j] = v;
    }
}

// The unitary circulant's first column (Section 6, Example exunc, real form):
// pairing u_j e^{-2 pi i jk/n} with its conjugate partner u_{n-j} gives
//   c_k = (s_0 + (-1)^k s_{n/2} + 2 sum_{0<j<n/2} cos(2 pi (phi_j - (jk mod n)/n))) / n,
// (s_{n/2} only for even n).  One thread a column entry; the phases pass
// through LDS in chunks of 1024.
__global__ __launch_bounds__(256) void k_unitary_column(const double *__restrict__ phi, int n,
                                                        double *__restrict__ c) {
    __shared__ double sp[1024];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int jmax = (n - 1) / 2;  // pairs j = 1 .. jmax
    const double inv_n = 1.0 / static_cast<double>(n);
    double acc = 0.0;
    for (int j0 = 1; j0 <= jmax; j0 += 1024) {
        const int cnt = min(1024, jmax - j0 + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) sp[t] = phi[j0 + t];
        __syncthreads();
        if (k < n) {
            int t = static_cast<int>((static_cast<int64_t>(j0) * k) % n);  // (j k) mod n
            for (int q = 0; q < cnt; ++q) {
                acc += cospi(2.0 * sp[q] - 2.0 * static_cast<double>(t) * inv_n);
                t += k;
                if (t >= n) t -= n;
            }
        }
    }
    if (k >= n) return;
    double v = 2.0 * acc + (phi[0] < 0.5 ? 1.0 : -1.0);
    if (n % 2 == 0) v += ((k & 1) ? -1.0 : 1.0) * (phi[n / 2] < 0.5 ? 1.0 : -1.0);
    c[k] = v * inv_n;
}

// The unitary circulant's half spectrum straight from its phases, for the
// period m = n (a power of two).  Pairing u_f = e^{2 pi i phi_f} with its
// conjugate partner as in the column formula above (Section 6, Example exunc)
// makes the column c = (1/n) sum_f u_f e^{-2 pi i f k / n}, whose DFT is
// conj(u_f): hhat_f = e^{-2 pi i phi_f} for 0 < f < n/2, and the real
// hhat_0 = s_0, hhat_{n/2} = s_{n/2} (+1 for a phase below 1/2, else -1).
__global__ __launch_bounds__(256) void k_unitary_spectrum(const double *__restrict__ phi, int L,
                                                          cplx *__restrict__ hhat) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f <= L; f += gridDim.x * blockDim.x) {
        if (f == 0 || f == L) {
            hhat[f] = {phi[f] < 0.5 ? 1.0 : -1.0, 0.0};
        } else {
            double sn, cs;
            sincospi(2.0 * phi[f], &sn, &cs);
            hhat[f] = {cs, -sn};
        }
    }
}

// ---------------------------------------------------------------- batches
// Circulant multipliers of many systems (n_s <= 1024, so m_s <= 2048 and a
// row fits one wave).  logl[s] = log2(m_s / 2); the twiddle table of period
// 2 L sits at tw_pool + tw_off[log2 L]; h and its half spectrum of system s at
// h_pool + h_off[s] (m_s doubles) and hh_pool + hh_off[s] (L_s + 1 complex).
template <int LG, typename TI, typename TO>
__device__ inline void batch_row(const TI *x, int64_t n, const cplx *tw, const cplx *hh, int conj,
                                 TO *y, cplx *spec, cplx *sm) {
    fft_row<LG, TI, TO>(x, 1, n, tw, hh, conj, 0.0, y, 1, spec, nullptr, sm);
}

template <typename TI, typename TO>
__device__ __attribute__((always_inline)) inline void batch_row_any(int lg, const TI *x, int64_t n, const cplx *tw,
                                     const cplx *hh, int conj, TO *y, cplx *spec, cplx *sm) {
    switch (lg) {
    case 0: batch_row<0, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 1: batch_row<1, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 2: batch_row<2, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 3: batch_row<3, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 4: batch_row<4, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 5: batch_row<5, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 6: batch_row<6, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 7: batch_row<7, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 8: batch_row<8, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    case 9: batch_row<9, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    default: batch_row<10, TI, TO>(x, n, tw, hh, conj, y, spec, sm); break;
    }
}

// One workgroup per circulant system: the period-m kernel h from the first
// column c (at c_pool + c_off[s]; as k_embed does for one circulant), then its
// half spectrum.
__global__ __launch_bounds__(64) void k_batch_spectrum(
    const int *__restrict__ nsys, const int *__restrict__ logl, const int64_t *__restrict__ c_off,
    const int64_t *__restrict__ h_off, const int64_t *__restrict__ hh_off,
    const int64_t *__restrict__ tw_off, const double *c_pool, double *h_pool, cplx *hh_pool,
    const cplx *tw_pool) {
    extern __shared__ cplx sm[];
    const int s = blockIdx.x, n = nsys[s], lg = logl[s], m = 2 << lg;
    const double *c = c_pool + c_off[s];
    double *h = h_pool + h_off[s];
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        double v = 0.0;
        if (m == n || j < n)
            v = c[j];
        else if (j > m - n)
            v = c[n - (m - j)];
        h[j] = v;
    }
    __syncthreads();
    batch_row_any<double, double>(lg, h, m, tw_pool + tw_off[lg], nullptr, 0,
                                  static_cast<double *>(nullptr), hh_pool + hh_off[s], sm);
}

// Rows of the products M_s = A_s C_s of all circulant systems: row r of the
// flattened row space (row_start: prefix sums of n_s) is row r - row_start[s]
// of system s; A in FP64, M in FP32 (the batch's factors) or FP64 (the
// fallback), both ld = n_s.  With flag != null only the systems whose flag
// (flag[sys[s]]) is set are done; the other rows' workgroups return at once.
template <typename TO>
__global__ __launch_bounds__(64) void k_batch_fft_rows(
    int count, const int *__restrict__ row_start, const int *__restrict__ nsys,
    const int *__restrict__ sys, const int *__restrict__ flag, const int *__restrict__ logl,
    const int64_t *__restrict__ a_off, const int64_t *__restrict__ m_off,
    const int64_t *__restrict__ hh_off, const int64_t *__restrict__ tw_off, const double *A,
    const cplx *hh_pool, const cplx *tw_pool, TO *M) {
    extern __shared__ cplx sm[];
    const int r = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= r) lo = mid; else hi = mid - 1;
    }
    const int s = lo;
    if (flag != nullptr && flag[sys[s]] == 0) return;
    const int n = nsys[s], lg = logl[s];
    const int64_t i = r - row_start[s];
    batch_row_any<double, TO>(lg, A + a_off[s] + i * n, n, tw_pool + tw_off[lg],
                              hh_pool + hh_off[s], 1, M + m_off[s] + i * n, nullptr, sm);
}

int log2i(int L) {
    int l = 0;
    while ((1 << l) < L) ++l;
    return l;
}


template <int LOGL, typename TI, typename TO>
hipError_t launch_stockham(const TI *in, int64_t vsi, int64_t esi, int64_t count, int64_t n,
                           const cplx *tw, const cplx *hhat, int conj, double beta, TO *out,
                           int64_t vso, int64_t eso, cplx *spec, double *absmax, hipStream_t s) {
    constexpr int L = 1 << LOGL;
    const size_t lds = sizeof(cplx) * static_cast<size_t>(L + L / 16 + 1);
    const int threads = L / 16 > 64 ? L / 16 : 64;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_stockham<LOGL, TI, TO>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fft_stockham<LOGL, TI, TO>), dim3(static_cast<unsigned>(count)),
                       dim3(threads), lds, s, in, vsi, esi, n, tw, hhat, conj, beta, out, vso, eso,
                       spec, absmax);
    return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_rows(const TI *in, int64_t vsi, int64_t esi, int64_t count, int64_t n, int m,
                       const cplx *tw, const cplx *hhat, int conj, double beta, TO *out,
                       int64_t vso, int64_t eso, cplx *spec, double *absmax, hipStream_t s) {
    if (count > 0x7fffffff) return hipErrorInvalidValue;
#define RMGE_FFT_CASE(LG)                                                                      \
    case LG:                                                                                   \
        return launch_stockham<LG, TI, TO>(in, vsi, esi, count, n, tw, hhat, conj, beta, out, \
                                           vso, eso, spec, absmax, s);
    switch (log2i(m / 2)) {
        RMGE_FFT_CASE(0) RMGE_FFT_CASE(1) RMGE_FFT_CASE(2) RMGE_FFT_CASE(3) RMGE_FFT_CASE(4)
        RMGE_FFT_CASE(5) RMGE_FFT_CASE(6) RMGE_FFT_CASE(7) RMGE_FFT_CASE(8) RMGE_FFT_CASE(9)
        RMGE_FFT_CASE(10) RMGE_FFT_CASE(11) RMGE_FFT_CASE(12) RMGE_FFT_CASE(13)
    default: return hipErrorInvalidValue;
    }
#undef RMGE_FFT_CASE
}

bool valid_m(int m) { return m >= 2 && m <= 16384 && (m & (m - 1)) == 0; }

}  // namespace

hipError_t fft_twiddles(int m, double *tw, hipStream_t s) {
    if (!valid_m(m)) return hipErrorInvalidValue;
    const int L = m / 2;
    hipLaunchKernelGGL(k_twiddles, dim3((L + 256) / 256), dim3(256), 0, s, L,
                       reinterpret_cast<cplx *>(tw));
    return hipGetLastError();
}

hipError_t unitary_spectrum(const double *phi, int64_t n, double *hhat, hipStream_t s) {
    if (n < 2 || n > 16384 || (n & (n - 1)) != 0) return hipErrorInvalidValue;
    const int L = static_cast<int>(n / 2);
    hipLaunchKernelGGL(k_unitary_spectrum, dim3(static_cast<unsigned>((L + 256) / 256)), dim3(256),
                       0, s, phi, L, reinterpret_cast<cplx *>(hhat));
    return hipGetLastError();
}

hipError_t unitary_column(const double *phi, int64_t n, double *c, hipStream_t s) {
    if (n < 1 || n > (int64_t(1) << 20)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_unitary_column, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       s, phi, static_cast<int>(n), c);
    return hipGetLastError();
}

hipError_t batch_fft_spectra(int count, const int *nsys, const int *logl, const int64_t *c_off,
                             const int64_t *h_off, const int64_t *hh_off, const int64_t *tw_off,
                             const double *c_pool, double *h_pool, double *hh_pool,
                             const double *tw_pool, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const size_t lds = sizeof(cplx) * (1024 + 64 + 1);
    hipLaunchKernelGGL(k_batch_spectrum, dim3(static_cast<unsigned>(count)), dim3(64), lds, s, nsys,
                       logl, c_off, h_off, hh_off, tw_off, c_pool, h_pool,
                       reinterpret_cast<cplx *>(hh_pool), reinterpret_cast<const cplx *>(tw_pool));
    return hipGetLastError();
}

template <typename TO>
hipError_t batch_fft_rows(int count, int total_rows, const int *row_start, const int *nsys,
                          const int *sys, const int *flag, const int *logl, const int64_t *a_off,
                          const int64_t *m_off, const int64_t *hh_off, const int64_t *tw_off,
                          const double *A, const double *hh_pool, const double *tw_pool, TO *M,
                          hipStream_t s) {
    if (count <= 0 || total_rows <= 0) return hipSuccess;
    const size_t lds = sizeof(cplx) * (1024 + 64 + 1);
    hipLaunchKernelGGL(k_batch_fft_rows<TO>, dim3(static_cast<unsigned>(total_rows)), dim3(64),
                       lds, s, count, row_start, nsys, sys, flag, logl, a_off, m_off, hh_off,
                       tw_off, A, reinterpret_cast<const cplx *>(hh_pool),
                       reinterpret_cast<const cplx *>(tw_pool), M);
    return hipGetLastError();
}

template hipError_t batch_fft_rows<float>(int, int, const int *, const int *, const int *,
                                          const int *, const int *, const int64_t *,
                                          const int64_t *, const int64_t *, const int64_t *,
                                          const double *, const double *, const double *, float *,
                                          hipStream_t);
template hipError_t batch_fft_rows<double>(int, int, const int *, const int *, const int *,
                                           const int *, const int *, const int64_t *,
                                           const int64_t *, const int64_t *, const int64_t *,
                                           const double *, const double *, const double *,
                                           double *, hipStream_t);

hipError_t fft_embed(int kind, const double *params, int64_t n, int m, double *h, hipStream_t s) {
    if (!valid_m(m)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_embed, dim3((m + 255) / 256), dim3(256), 0, s, kind, params, n, m, h);
    return hipGetLastError();
}

hipError_t fft_spectrum(const double *h, int m, const double *tw, double *hhat, hipStream_t s) {
    if (!valid_m(m)) return hipErrorInvalidValue;
    return launch_rows<double, double>(h, 0, 1, 1, m, m, reinterpret_cast<const cplx *>(tw),
                                       nullptr, 0, 0.0, static_cast<double *>(nullptr), 0, 0,
                                       reinterpret_cast<cplx *>(hhat), nullptr, s);
}

template <typename TI, typename TO>
hipError_t fft_rows(const TI *in, int64_t vstride_in, int64_t estride_in, int64_t count,
                    int64_t n, int m, const double *tw, const double *hhat, int conj, double beta,
                    TO *out, int64_t vstride_out, int64_t estride_out, hipStream_t s,
                    double *absmax) {
    if (count <= 0) return hipSuccess;
    if (!valid_m(m) || n > m) return hipErrorInvalidValue;
    return launch_rows<TI, TO>(in, vstride_in, estride_in, count, n, m,
                               reinterpret_cast<const cplx *>(tw),
                               reinterpret_cast<const cplx *>(hhat), conj, beta, out, vstride_out,
                               estride_out, nullptr, absmax, s);
}

template hipError_t fft_rows<double, double>(const double *, int64_t, int64_t, int64_t, int64_t,
                                             int, const double *, const double *, int, double,
                                             double *, int64_t, int64_t, hipStream_t, double *);
template hipError_t fft_rows<double, float>(const double *, int64_t, int64_t, int64_t, int64_t,
                                            int, const double *, const double *, int, double,
                                            float *, int64_t, int64_t, hipStream_t, double *);
template hipError_t fft_rows<float, double>(const float *, int64_t, int64_t, int64_t, int64_t, int,
                                            const double *, const double *, int, double, double *,
                                            int64_t, int64_t, hipStream_t, double *);

}  // namespace rmge
