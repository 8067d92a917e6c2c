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
// z_k = x_{2k} + i x_{2k+1} (k < L = m/2) and transformed with an in-place
// radix-2 complex FFT of length L in LDS (decimation in time from bit-reversed
// order, natural-order spectrum); the real spectrum is untangled pairwise
// (f, L - f), multiplied by the kernel's spectrum, re-packed, and sent back
// through a decimation-in-frequency inverse whose bit-reversed output is read
// directly when storing.  Twiddles e^{-i pi j / L}, j = 0..L, come from a table
// built once per multiplier.
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

__device__ inline int bitrev(int k, int logL) {
    return logL == 0 ? 0 : static_cast<int>(__brev(static_cast<unsigned>(k)) >> (32 - logL));
}

__global__ void k_twiddles(int L, cplx *tw) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j <= L; j += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-static_cast<double>(j) / static_cast<double>(L), &s, &c);
        tw[j] = {c, s};
    }
}

// Forward transform of a real vector of length m (zero padded from n).  If
// spec != null the half spectrum X_0..X_L is written there and the kernel ends.
// Otherwise Y = X * K (K = conj(hhat) if conj) is inverted and
// out = beta * out + y[0..n).
template <typename TI, typename TO>
__global__ __launch_bounds__(1024) void k_fft_rows(const TI *in, int64_t vsi, int64_t esi,
                                                   int64_t n, int L, int logL, const cplx *tw,
                                                   const cplx *hhat, int conj, double beta, TO *out,
                                                   int64_t vso, int64_t eso, cplx *spec,
                                                   double *absmax) {
    extern __shared__ cplx z[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t v = blockIdx.x;
    const TI *x = in + v * vsi;
    for (int k = tid; k < L; k += nt) {
        const int64_t j0 = 2 * static_cast<int64_t>(k), j1 = j0 + 1;
        const double re = j0 < n ? static_cast<double>(x[j0 * esi]) : 0.0;
        const double im = j1 < n ? static_cast<double>(x[j1 * esi]) : 0.0;
        z[bitrev(k, logL)] = {re, im};
    }
    __syncthreads();
    for (int h = 1; h < L; h <<= 1) {  // decimation in time
        const int stride = L / h;
        for (int t = tid; t < L / 2; t += nt) {
            const int pos = t & (h - 1);
            const int i0 = ((t - pos) << 1) + pos, i1 = i0 + h;
            const cplx u = z[i0], b = cmul(z[i1], tw[pos * stride]);
            z[i0] = u + b;
            z[i1] = u - b;
        }
        __syncthreads();
    }
    // Pairs (f, L - f): untangle the real spectrum, apply the kernel, re-pack.
    for (int f = tid; f <= L / 2; f += nt) {
        const int g = (L - f) & (L - 1);
        const cplx Zf = z[f], Zg = z[g];
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
        z[f] = {ep.x - op.y, ep.y + op.x};  // E' + i O'
        if (f != 0 && g != f) {
            const cplx ec = cconj(ep), oc = cconj(op);
            z[g] = {ec.x - oc.y, ec.y + oc.x};
        }
    }
    if (spec != nullptr) return;
    __syncthreads();
    for (int h = L / 2; h >= 1; h >>= 1) {  // decimation in frequency, inverse sign
        const int stride = L / h;
        for (int t = tid; t < L / 2; t += nt) {
            const int pos = t & (h - 1);
            const int i0 = ((t - pos) << 1) + pos, i1 = i0 + h;
            const cplx u = z[i0], b = z[i1];
            z[i0] = u + b;
            z[i1] = cmul(u - b, cconj(tw[pos * stride]));
        }
        __syncthreads();
    }
    const double scale = 1.0 / static_cast<double>(L);
    TO *y = out + v * vso;
    double vmax = 0.0;
    for (int k = tid; k < L; k += nt) {
        const cplx zz = z[bitrev(k, logL)];
        const int64_t j0 = 2 * static_cast<int64_t>(k), j1 = j0 + 1;
        if (j0 < n) {
            TO *p = y + j0 * eso;
            const double val = zz.x * scale;
            const TO o = static_cast<TO>(beta == 0.0 ? val : beta * static_cast<double>(*p) + val);
            *p = o;
            vmax = fmax(vmax, fabs(static_cast<double>(o)));
        }
        if (j1 < n) {
            TO *p = y + j1 * eso;
            const double val = zz.y * scale;
            const TO o = static_cast<TO>(beta == 0.0 ? val : beta * static_cast<double>(*p) + val);
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

int log2i(int L) {
    int l = 0;
    while ((1 << l) < L) ++l;
    return l;
}

int fft_threads(int L) {
    int t = L / 8;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

template <typename TI, typename TO>
hipError_t launch_rows(const TI *in, int64_t vsi, int64_t esi, int64_t count, int64_t n, int m,
                       const cplx *tw, const cplx *hhat, int conj, double beta, TO *out,
                       int64_t vso, int64_t eso, cplx *spec, double *absmax, hipStream_t s) {
    const int L = m / 2;
    const size_t lds = sizeof(cplx) * static_cast<size_t>(L);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_rows<TI, TO>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fft_rows<TI, TO>), dim3(static_cast<unsigned>(count)),
                       dim3(fft_threads(L)), lds, s, in, vsi, esi, n, L, log2i(L), tw, hhat, conj,
                       beta, out, vso, eso, spec, absmax);
    return hipGetLastError();
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
