/*
 * rta_oracle.c -- FP64 CPU oracle for multichannel (MIMO) FIR convolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the benchmark's
 * CPU-baseline leg can compare the GPU library against a plain, slow and
 * obviously correct computation of what the partitioned convolution must
 * produce.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper: Sec. III-A Eq. 1-2, Sec. III-B Eq. 4-5, Sec. IV):
 *
 *   y_l[n] = sum_{q=0}^{Q-1} sum_{j=0}^{n_h(q,l)-1} h_{ql}[j] * x_q[n-j],
 *   with x_q[m] = 0 for m < 0 and for m >= n_x.
 *
 * Uniform and non-uniform partitioned overlap-save (UPOLS / NUPC) only
 * regroup this sum, so both reach exactly this result up to rounding; the
 * oracle is therefore the definition itself (direct form, Eq. 4 summed over
 * inputs as in Eq. 2) plus one plain FFT overlap-save form (Eq. 5 applied to
 * successive input segments, keeping only the samples that are free of
 * circular wrap-around, Sec. IV step 3).  Indices are 0-based and causal: an
 * impulse at n = 0 returns the filter itself.
 *
 * Filters are passed as one concatenated array `h` with offsets `off` of
 * length Q*L+1; pair (q,l) -- row-major [in][out], the Q x L matrix H of
 * Eq. 1 -- occupies h[off[q*L+l] .. off[q*L+l+1]).  A zero-length pair has
 * no path.  Signals are row-major [channel][sample].  All arithmetic is in
 * IEEE double; the build uses -ffp-contract=off so no FMA contraction
 * changes rounding between compilers.
 *
 * Feedback-cancellation loop (Sec. III-A Eq. 3 and Sec. V, the paper's
 * auralization step): with P microphone signals m_p, synthesis filters
 * h_pl (P x L, the H of Eq. 1) and estimated feedback paths f_pl (P x L,
 * the F-hat of Eq. 3, path from loudspeaker l to microphone p), block by
 * block of B samples
 *     mt_p[t] = m_p[t] - c_p[t - B]          (c_p[t] = 0 for t < 0)
 *     l_l[t]  = sum_p sum_j h_pl[j] mt_p[t - j]
 *     c_p[t]  = sum_l sum_j f_pl[j] l_l[t - j]
 * i.e. the feedback estimate of one block is subtracted from the next block
 * of microphone samples.  Every sum is the direct form above.
 *
 * Serving with feedback cancellation (the same loop with sources that come
 * and go; a reading of Sec. III-A Eq. 1-3 and Sec. V for a system whose
 * talkers change): Q microphone slots with fixed feedback paths f_ql, and
 * sources s, each bound to one slot q_s, live during blocks [a_s, b_s)
 * (one source per slot at a time) and carrying its own filter row h_sl.
 * Per block n, for t in [nB, (n+1)B):
 *     mt_q[t] = m_q[t] - c_q[t - B]   if a source of slot q is live in n,
 *               0                      otherwise;
 *     x_s[t]  = mt_{q_s}[t] if a_s <= n < b_s, else 0;
 *     l_l[t]  = sum_s sum_j h_sl[j] x_s[t - j];
 *     c_q[t]  = sum_l sum_j f_ql[j] l_l[t - j].
 * A source that has left keeps ringing through its own filters (its input
 * is zero from b_s on); with every slot live throughout and h_sl the row of
 * slot q_s, this is the loop above.
 *
 * Return codes: 0 on success, -1 on an invalid argument, -2 if memory for
 * the FFT work buffers cannot be allocated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Threads the OpenMP loops below run on (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int valid_layout(int Q, int L, const int64_t* off) {
    if (Q <= 0 || L <= 0 || off == NULL) return 0;
    if (off[0] != 0) return 0;
    for (int64_t i = 0; i < (int64_t)Q * L; ++i)
        if (off[i + 1] < off[i]) return 0;
    return 1;
}

/* One output sample of one (q,l) pair, Eq. 4 with 0-based causal indices:
 * sum over the filter taps j whose input index n-j lies inside [0, n_x). */
static double pair_sample(const double* x, int64_t nx, const double* h,
                          int64_t nh, int64_t n) {
    double s = 0.0;
    for (int64_t j = 0; j < nh; ++j) {
        int64_t m = n - j;
        if (m < 0) break;         /* taps are visited in increasing j */
        if (m >= nx) continue;    /* input not yet started / already over */
        s += h[j] * x[m];
    }
    return s;
}

/* Eq. 2: output l at sample n, summed over the inputs q in order. */
static double mimo_sample(int Q, int L, const double* x, int64_t nx,
                          const double* h, const int64_t* off, int l,
                          int64_t n) {
    double s = 0.0;
    for (int q = 0; q < Q; ++q) {
        int64_t pi = (int64_t)q * L + l;
        s += pair_sample(x + (int64_t)q * nx, nx, h + off[pi],
                         off[pi + 1] - off[pi], n);
    }
    return s;
}

/* Direct form over the contiguous output range [n0, n1):
 * y is [L][n1-n0]. */
int orc_direct_range(int Q, int L, const double* x, int64_t nx,
                     const double* h, const int64_t* off, int64_t n0,
                     int64_t n1, double* y) {
    if (!valid_layout(Q, L, off) || x == NULL || y == NULL || nx < 0 ||
        n1 < n0)
        return -1;
    int64_t ny = n1 - n0;
    int64_t total = (int64_t)L * ny;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < total; ++t) {
        int l = (int)(t / ny);
        int64_t i = t % ny;
        y[t] = mimo_sample(Q, L, x, nx, h, off, l, n0 + i);
    }
    return 0;
}

/* Direct form at an arbitrary list of output indices: y is [L][n_idx],
 * y[l][i] = y_l[idx[i]].  Used for spot checks at full problem sizes. */
int orc_direct_at(int Q, int L, const double* x, int64_t nx, const double* h,
                  const int64_t* off, const int64_t* idx, int64_t n_idx,
                  double* y) {
    if (!valid_layout(Q, L, off) || x == NULL || y == NULL || idx == NULL ||
        nx < 0 || n_idx < 0)
        return -1;
    int64_t total = (int64_t)L * n_idx;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < total; ++t) {
        int l = (int)(t / n_idx);
        int64_t i = t % n_idx;
        y[t] = mimo_sample(Q, L, x, nx, h, off, l, idx[i]);
    }
    return 0;
}

/* In-place iterative radix-2 complex DFT of length n (a power of two):
 *   X[k] = sum_m z[m] exp(sign * 2*pi*i*k*m/n),  unnormalized.
 * sign = -1 is the forward transform of Eq. 5, +1 the inverse without the
 * 1/n factor.  Every twiddle is evaluated directly as cos/sin of its own
 * angle (no recurrence), once per stage. */
int orc_fft(double* re, double* im, int64_t n, int sign) {
    if (re == NULL || im == NULL || n < 1 || (n & (n - 1)) != 0 ||
        (sign != 1 && sign != -1))
        return -1;
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = re[i]; re[i] = re[j]; re[j] = tr;
            double ti = im[i]; im[i] = im[j]; im[j] = ti;
        }
    }
    double* wr = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    double* wi = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    if (wr == NULL || wi == NULL) { free(wr); free(wi); return -2; }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len / 2;
        for (int64_t k = 0; k < half; ++k) {
            double ang = (double)sign * 2.0 * M_PI * (double)k / (double)len;
            wr[k] = cos(ang);
            wi[k] = sin(ang);
        }
        for (int64_t s = 0; s < n; s += len) {
            for (int64_t k = 0; k < half; ++k) {
                int64_t a = s + k, b = s + k + half;
                double br = re[b] * wr[k] - im[b] * wi[k];
                double bi = re[b] * wi[k] + im[b] * wr[k];
                re[b] = re[a] - br;
                im[b] = im[a] - bi;
                re[a] = re[a] + br;
                im[a] = im[a] + bi;
            }
        }
    }
    free(wr);
    free(wi);
    return 0;
}

/* Single-partition FFT overlap-save (Eq. 5 per segment, Sec. IV step 3):
 *   M = smallest power of two >= 2*N_h (N_h = longest filter, at least 1),
 *   hop S = M - N_h + 1.  Segment s covers outputs [s*S, s*S+S); its input
 *   window is x_q[s*S-(N_h-1) + i], i in [0,M) (zero outside the signal).
 *   Y_l = sum_q FFT(h_ql zero-padded to M) .* FFT(window_q)  (Eq. 2, 5),
 *   and IFFT(Y_l)/M at positions [N_h-1, M) are linear-convolution samples.
 * y is [L][n_y] and receives y_l[0 .. n_y). */
int orc_fftols(int Q, int L, const double* x, int64_t nx, const double* h,
               const int64_t* off, int64_t ny, double* y) {
    if (!valid_layout(Q, L, off) || x == NULL || y == NULL || nx < 0 ||
        ny < 0)
        return -1;
    int64_t nh = 1;
    for (int64_t p = 0; p < (int64_t)Q * L; ++p)
        if (off[p + 1] - off[p] > nh) nh = off[p + 1] - off[p];
    int64_t M = 2;
    while (M < 2 * nh) M <<= 1;
    int64_t S = M - nh + 1;
    int64_t nseg = (ny + S - 1) / S;

    /* spectra of the Q input windows of one segment, shared by all outputs */
    double* wre = (double*)malloc(sizeof(double) * (size_t)(Q * M));
    double* wim = (double*)malloc(sizeof(double) * (size_t)(Q * M));
    if (wre == NULL || wim == NULL) { free(wre); free(wim); return -2; }
    int status = 0;

    for (int64_t s = 0; s < nseg && status == 0; ++s) {
        int64_t start = s * S - (nh - 1);
#pragma omp parallel for schedule(static)
        for (int q = 0; q < Q; ++q) {
            double* r = wre + (int64_t)q * M;
            double* im = wim + (int64_t)q * M;
            for (int64_t i = 0; i < M; ++i) {
                int64_t m = start + i;
                r[i] = (m >= 0 && m < nx) ? x[(int64_t)q * nx + m] : 0.0;
                im[i] = 0.0;
            }
            orc_fft(r, im, M, -1);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int l = 0; l < L; ++l) {
            double* yr = (double*)calloc((size_t)M, sizeof(double));
            double* yi = (double*)calloc((size_t)M, sizeof(double));
            double* hr = (double*)malloc(sizeof(double) * (size_t)M);
            double* hi = (double*)malloc(sizeof(double) * (size_t)M);
            if (yr == NULL || yi == NULL || hr == NULL || hi == NULL) {
#pragma omp atomic write
                status = -2;
                free(yr); free(yi); free(hr); free(hi);
                continue;
            }
            for (int q = 0; q < Q; ++q) {
                int64_t pi = (int64_t)q * L + l;
                int64_t len = off[pi + 1] - off[pi];
                if (len == 0) continue;
                for (int64_t i = 0; i < M; ++i) {
                    hr[i] = i < len ? h[off[pi] + i] : 0.0;
                    hi[i] = 0.0;
                }
                orc_fft(hr, hi, M, -1);
                const double* xr = wre + (int64_t)q * M;
                const double* xi = wim + (int64_t)q * M;
                for (int64_t k = 0; k < M; ++k) {
                    yr[k] += hr[k] * xr[k] - hi[k] * xi[k];
                    yi[k] += hr[k] * xi[k] + hi[k] * xr[k];
                }
            }
            orc_fft(yr, yi, M, +1);
            for (int64_t i = 0; i < S; ++i) {
                int64_t n = s * S + i;
                if (n >= ny) break;
                y[(int64_t)l * ny + n] = yr[nh - 1 + i] / (double)M;
            }
            free(yr); free(yi); free(hr); free(hi);
        }
    }
    free(wre);
    free(wim);
    return status;
}

/* Closed feedback-cancellation loop (see the file header).  m is [P][N];
 * h and f are P x L pair arrays with offsets hoff/foff (pair (p,l) at
 * index p*L+l); l_out is [L][N], c_out is [P][N], mt_out ([P][N]) may be
 * NULL.  The blocks are processed in order; within a block every output
 * sample only uses samples of the same or earlier blocks. */
int orc_feedback_loop(int P, int L, const double* m, int64_t N, int64_t B,
                      const double* h, const int64_t* hoff, const double* f,
                      const int64_t* foff, double* l_out, double* c_out,
                      double* mt_out) {
    if (!valid_layout(P, L, hoff) || !valid_layout(P, L, foff) || m == NULL ||
        l_out == NULL || c_out == NULL || N < 0 || B < 1)
        return -1;
    double* mt = mt_out;
    if (mt == NULL) {
        mt = (double*)malloc(sizeof(double) * (size_t)(P * N + 1));
        if (mt == NULL) return -2;
    }
    for (int64_t t0 = 0; t0 < N; t0 += B) {
        int64_t t1 = t0 + B < N ? t0 + B : N;
        for (int p = 0; p < P; ++p)
            for (int64_t t = t0; t < t1; ++t)
                mt[(int64_t)p * N + t] =
                    m[(int64_t)p * N + t] - (t >= B ? c_out[(int64_t)p * N + t - B] : 0.0);
#pragma omp parallel for schedule(static)
        for (int l = 0; l < L; ++l)
            for (int64_t t = t0; t < t1; ++t) {
                double s = 0.0;
                for (int p = 0; p < P; ++p) {
                    int64_t pi = (int64_t)p * L + l;
                    s += pair_sample(mt + (int64_t)p * N, t1, h + hoff[pi],
                                     hoff[pi + 1] - hoff[pi], t);
                }
                l_out[(int64_t)l * N + t] = s;
            }
#pragma omp parallel for schedule(static)
        for (int p = 0; p < P; ++p)
            for (int64_t t = t0; t < t1; ++t) {
                double s = 0.0;
                for (int l = 0; l < L; ++l) {
                    int64_t pi = (int64_t)p * L + l;
                    s += pair_sample(l_out + (int64_t)l * N, t1, f + foff[pi],
                                     foff[pi + 1] - foff[pi], t);
                }
                c_out[(int64_t)p * N + t] = s;
            }
    }
    if (mt_out == NULL) free(mt);
    return 0;
}

/* Serving loop with feedback cancellation (see the file header).  m is
 * [Q][N]; source s has slot src_slot[s], live blocks [src_a[s], src_b[s])
 * and filters h[hoff[s*L+l] .. hoff[s*L+l+1]) to output l; f is a Q x L
 * pair array with offsets foff.  l_out is [L][N], c_out and mt_out [Q][N]. */
int orc_serve_loop(int Q, int L, int S, const double* m, int64_t N, int64_t B,
                   const int32_t* src_slot, const int64_t* src_a, const int64_t* src_b,
                   const double* h, const int64_t* hoff, const double* f,
                   const int64_t* foff, double* l_out, double* c_out, double* mt_out) {
    if (Q <= 0 || L <= 0 || S < 0 || m == NULL || N < 0 || B < 1 || l_out == NULL ||
        c_out == NULL || mt_out == NULL || !valid_layout(Q, L, foff))
        return -1;
    if (S > 0 && (src_slot == NULL || src_a == NULL || src_b == NULL || !valid_layout(S, L, hoff)))
        return -1;
    for (int s = 0; s < S; ++s)
        if (src_slot[s] < 0 || src_slot[s] >= Q || src_b[s] < src_a[s]) return -1;
    /* x_s: the input each source sees */
    double* x = (double*)calloc((size_t)(S > 0 ? S : 1) * (size_t)(N > 0 ? N : 1), sizeof(double));
    if (x == NULL) return -2;
    for (int64_t t0 = 0; t0 < N; t0 += B) {
        const int64_t n = t0 / B;
        const int64_t t1 = t0 + B < N ? t0 + B : N;
        for (int q = 0; q < Q; ++q) {
            int live = 0;
            for (int s = 0; s < S; ++s)
                if (src_slot[s] == q && src_a[s] <= n && n < src_b[s]) live = 1;
            for (int64_t t = t0; t < t1; ++t)
                mt_out[(int64_t)q * N + t] =
                    live ? m[(int64_t)q * N + t] - (t >= B ? c_out[(int64_t)q * N + t - B] : 0.0)
                         : 0.0;
        }
        for (int s = 0; s < S; ++s) {
            const int on = src_a[s] <= n && n < src_b[s];
            for (int64_t t = t0; t < t1; ++t)
                x[(int64_t)s * N + t] = on ? mt_out[(int64_t)src_slot[s] * N + t] : 0.0;
        }
#pragma omp parallel for schedule(static)
        for (int l = 0; l < L; ++l)
            for (int64_t t = t0; t < t1; ++t) {
                double acc = 0.0;
                for (int s = 0; s < S; ++s) {
                    int64_t pi = (int64_t)s * L + l;
                    acc += pair_sample(x + (int64_t)s * N, t1, h + hoff[pi],
                                       hoff[pi + 1] - hoff[pi], t);
                }
                l_out[(int64_t)l * N + t] = acc;
            }
#pragma omp parallel for schedule(static)
        for (int q = 0; q < Q; ++q)
            for (int64_t t = t0; t < t1; ++t) {
                double acc = 0.0;
                for (int l = 0; l < L; ++l) {
                    int64_t pi = (int64_t)q * L + l;
                    acc += pair_sample(l_out + (int64_t)l * N, t1, f + foff[pi],
                                       foff[pi + 1] - foff[pi], t);
                }
                c_out[(int64_t)q * N + t] = acc;
            }
    }
    free(x);
    return 0;
}
