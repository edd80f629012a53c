// Inverse FFT of the oversampled grid, crop, and deapodization
// (the sum over psi_m = e^{2 pi i m x} / w(x) of eq:cgmatrix and zeta_n = psi_n / w
// of eq:newadm).
//
// The transform wanted is J[q] = sum_g H[g] e^{+2 pi i (g - G/2)(q - G/2)/G}
// for the centred n outputs q = p + (G - n)/2. With G divisible by 4,
// (g - G/2)(q - G/2)/G = gq/G - g/2 - q/2 + G/4, so J[q] = (-1)^q sum_g
// (-1)^g H[g] e^{2 pi i g q / G}: a plain unnormalised inverse DFT with sign
// flips on load and store.
//
// One workgroup transforms RB consecutive rows of length G, one after another
// in LDS (Stockham autosort, one radix-2 or radix-4 stage when log2 G is not
// a multiple of 3, then radix-8 stages; every stage reads its butterfly
// inputs into registers, synchronises, and writes in place). Only the n cropped outputs are kept,
// in registers, and stored transposed once all RB rows are done, so that each
// store is an RB-element (32-byte) segment and the next pass again reads
// contiguous rows:
//   pass 1: rows g0 of H (G x G)  -> T1[q1'][g0]  (n x G)
//   pass 2: rows q1' of T1         -> image[p0][p1] (n x n), times
//           1/Phi(x_p0/sigma) / Phi(x_p1/sigma) formed in float64.
// Row blocks are assigned so that each of the 8 XCDs (workgroups are dealt to
// XCDs round-robin) works on a contiguous range of rows; the 32-byte segments
// of neighbouring blocks then meet in that XCD's L2 and leave it as whole
// lines.
#include "ftcg_internal.h"
#include "batch_internal.h"

namespace ftcg {

template <class real>
struct CxF;
template <>
struct CxF<float> {
  using t = float2;
  static __device__ inline void sincospi_(float x, float* s, float* c) { sincospif(x, s, c); }
};
template <>
struct CxF<double> {
  using t = double2;
  static __device__ inline void sincospi_(double x, double* s, double* c) { sincospi(x, s, c); }
};

template <class cx>
__device__ inline cx cmul(cx a, cx b) {
  cx r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class cx>
__device__ inline cx cadd(cx a, cx b) {
  cx r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <class cx>
__device__ inline cx csub(cx a, cx b) {
  cx r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <class cx>
__device__ inline cx cmul_i(cx a) {  // a * (+i)
  cx r;
  r.x = -a.y;
  r.y = a.x;
  return r;
}

// inverse (positive exponent) DFT of 4 and of 8 points in registers
template <class cx>
__device__ inline void idft4(cx& a0, cx& a1, cx& a2, cx& a3) {
  const cx s0 = cadd(a0, a2), s1 = csub(a0, a2), s2 = cadd(a1, a3), s3 = cmul_i(csub(a1, a3));
  a0 = cadd(s0, s2);
  a1 = cadd(s1, s3);
  a2 = csub(s0, s2);
  a3 = csub(s1, s3);
}

template <class cx>
__device__ inline void idft8(cx (&v)[8]) {
  using real = decltype(v[0].x);
  // even and odd halves, then V[m] = E[m] + e^{i pi m / 4} O[m], V[m + 4] = E[m] - ...
  idft4(v[0], v[2], v[4], v[6]);
  idft4(v[1], v[3], v[5], v[7]);
  const real c = (real)0.70710678118654752440;
  cx o1, o2, o3;
  o1.x = (v[3].x - v[3].y) * c;
  o1.y = (v[3].x + v[3].y) * c;
  o2 = cmul_i(v[5]);
  o3.x = -(v[7].x + v[7].y) * c;
  o3.y = (v[7].x - v[7].y) * c;
  const cx e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], od0 = v[1];
  v[0] = cadd(e0, od0);
  v[4] = csub(e0, od0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// Row buffers in LDS are padded with one element after every 32 (element i
// at lp(i)): the first radix-8 stage writes at a stride of 8 elements, which
// without the pad puts 8 lanes of a half-wavefront on one bank.
__device__ inline int lp(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int padded_len(int L) { return L + (L >> 5); }

// in-place inverse (positive exponent) FFT of buf[0..L) in LDS, L = 2^log2L,
// by threads tid = 0..nth-1, nth >= L / PPT (PPT points per thread per
// stage, a multiple of 8); every thread of the workgroup calls it with the
// same L. Stockham autosort: one radix-2 or radix-4 stage when log2 L is not
// a multiple of 3, then radix-8 stages; a radix-R stage over spans Ns reads
// the R inputs b + r L/R of butterfly b into registers, multiplies input r by
// e^{2 pi i r k / (R Ns)} (k = b mod Ns), synchronises, and writes the R
// outputs to (b - k) R + k + m Ns. Twiddles: with w(j) = e^{2 pi i j /
// 2^log2T} (2^log2T >= L), e^{2 pi i k / (8 Ns)} = w(k << (log2T - log2(8
// Ns))), and w(j) = hi[j >> 6] * lo[j & 63] from the two LDS tables lo[t] =
// w(t), hi[t] = w(64 t) (both formed in float64); the other six twiddles of
// a radix-8 butterfly are its powers 2 .. 7, each at most three products
// from the first.
template <class real, int PPT>
__device__ __attribute__((always_inline)) inline void lds_ifft(typename CxF<real>::t* buf, int L, int log2L, int tid, int nth,
                         const typename CxF<real>::t* tw_lo, const typename CxF<real>::t* tw_hi, int log2T) {
  using cx = typename CxF<real>::t;
  static_assert(PPT % 8 == 0, "radix-8 stages take 8 points per butterfly");
  int Ns = 1, log2Ns = 0;
  const int pre = log2L % 3;
  if (pre == 1) {
    // radix 2, Ns = 1: no twiddles
    constexpr int NB = PPT / 2;
    cx v0[NB], v1[NB];
    const int half = L >> 1;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (tid + u * nth < half) {
        const int b = tid + u * nth;
        v0[u] = buf[lp(b)];
        v1[u] = buf[lp(b + half)];
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (tid + u * nth < half) {
        const int b = tid + u * nth;
        buf[lp(2 * b)] = cadd(v0[u], v1[u]);
        buf[lp(2 * b + 1)] = csub(v0[u], v1[u]);
      }
    __syncthreads();
    Ns = 2;
    log2Ns = 1;
  } else if (pre == 2) {
    // radix 4, Ns = 1: no twiddles
    constexpr int NB = PPT / 4;
    cx v[NB][4];
    const int quarter = L >> 2;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (tid + u * nth < quarter) {
        const int b = tid + u * nth;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[u][r] = buf[lp(b + r * quarter)];
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (tid + u * nth < quarter) {
        const int b = tid + u * nth;
        idft4(v[u][0], v[u][1], v[u][2], v[u][3]);
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[lp(4 * b + r)] = v[u][r];
      }
    __syncthreads();
    Ns = 4;
    log2Ns = 2;
  }
  constexpr int NB8 = PPT / 8;
  const int eighth = L >> 3;
  for (; Ns < L; Ns <<= 3, log2Ns += 3) {
    const int sh = log2T - log2Ns - 3;
    cx v[NB8][8];
#pragma unroll
    for (int u = 0; u < NB8; ++u)
      if (tid + u * nth < eighth) {
        const int b = tid + u * nth;
        const int k = b & (Ns - 1);
#pragma unroll
        for (int r = 0; r < 8; ++r) v[u][r] = buf[lp(b + r * eighth)];
        if (Ns > 1) {
          const int j = k << sh;
          const cx w1 = cmul(tw_hi[j >> 6], tw_lo[j & 63]);
          const cx w2 = cmul(w1, w1);
          const cx w3 = cmul(w2, w1);
          const cx w4 = cmul(w2, w2);
          v[u][1] = cmul(v[u][1], w1);
          v[u][2] = cmul(v[u][2], w2);
          v[u][3] = cmul(v[u][3], w3);
          v[u][4] = cmul(v[u][4], w4);
          v[u][5] = cmul(v[u][5], cmul(w4, w1));
          v[u][6] = cmul(v[u][6], cmul(w4, w2));
          v[u][7] = cmul(v[u][7], cmul(w4, w3));
        }
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB8; ++u)
      if (tid + u * nth < eighth) {
        const int b = tid + u * nth;
        const int k = b & (Ns - 1);
        idft8(v[u]);
        const int d = (b - k) * 8 + k;
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[lp(d + r * Ns)] = v[u][r];
      }
    __syncthreads();
  }
}

// A row of L = PPT * nts points held in registers, thread t holding v[u] =
// element t + u nts, transformed through two LDS buffers. The first
// butterflies of a thread (b = t + u nts, inputs b + r L/R) read only its own
// elements, and so do the outputs of its last radix-8 butterflies (written to
// b + r L/8), so the first stage is taken from the registers the row was
// loaded into and the last one leaves its outputs there: on return v[u] holds
// output element t + u nts. In between the stages run out of place (read one
// buffer, write the other), one barrier each, and the row makes 4 LDS round
// trips and 4 barriers at L = 8192 instead of 6 and 12. The buffer the last
// stage read may still be read by slower threads on return, so the next row
// starts in the other one (cur names the buffer the next first stage
// writes). Twiddles as in lds_ifft.
template <class real, int PPT>
__device__ __attribute__((always_inline)) inline void reg_ifft_db(typename CxF<real>::t (&v)[PPT],
                                                                  typename CxF<real>::t* b0,
                                                                  typename CxF<real>::t* b1, int& cur, int L,
                                                                  int log2L, int t, int nts,
                                                                  const typename CxF<real>::t* tw_lo,
                                                                  const typename CxF<real>::t* tw_hi, int log2T) {
  using cx = typename CxF<real>::t;
  static_assert(PPT % 8 == 0, "radix-8 stages take 8 points per butterfly");
  cx* A = cur ? b1 : b0;
  cx* B = cur ? b0 : b1;
  int Ns, log2Ns;
  const int pre = log2L % 3;
  if (pre == 1) {
    constexpr int NB = PPT / 2;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int b = t + u * nts;
      A[lp(2 * b)] = cadd(v[u], v[u + NB]);
      A[lp(2 * b + 1)] = csub(v[u], v[u + NB]);
    }
    Ns = 2;
    log2Ns = 1;
  } else if (pre == 2) {
    constexpr int NB = PPT / 4;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int b = t + u * nts;
      cx w0 = v[u], w1 = v[u + NB], w2 = v[u + 2 * NB], w3 = v[u + 3 * NB];
      idft4(w0, w1, w2, w3);
      A[lp(4 * b)] = w0;
      A[lp(4 * b + 1)] = w1;
      A[lp(4 * b + 2)] = w2;
      A[lp(4 * b + 3)] = w3;
    }
    Ns = 4;
    log2Ns = 2;
  } else {
    constexpr int NB = PPT / 8;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int b = t + u * nts;
      cx w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = v[u + r * NB];
      idft8(w);
#pragma unroll
      for (int r = 0; r < 8; ++r) A[lp(8 * b + r)] = w[r];
    }
    Ns = 8;
    log2Ns = 3;
  }
  constexpr int NB8 = PPT / 8;
  const int eighth = L >> 3;
  auto twiddle = [&](cx (&w)[8], int k, int sh) {
    const int j = k << sh;
    const cx w1 = cmul(tw_hi[j >> 6], tw_lo[j & 63]);
    const cx w2 = cmul(w1, w1);
    const cx w3 = cmul(w2, w1);
    const cx w4 = cmul(w2, w2);
    w[1] = cmul(w[1], w1);
    w[2] = cmul(w[2], w2);
    w[3] = cmul(w[3], w3);
    w[4] = cmul(w[4], w4);
    w[5] = cmul(w[5], cmul(w4, w1));
    w[6] = cmul(w[6], cmul(w4, w2));
    w[7] = cmul(w[7], cmul(w4, w3));
  };
  for (; Ns < eighth; Ns <<= 3, log2Ns += 3) {
    __syncthreads();
    const int sh = log2T - log2Ns - 3;
#pragma unroll
    for (int u = 0; u < NB8; ++u) {
      const int b = t + u * nts;
      const int k = b & (Ns - 1);
      cx w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = A[lp(b + r * eighth)];
      twiddle(w, k, sh);
      idft8(w);
      const int d = (b - k) * 8 + k;
#pragma unroll
      for (int r = 0; r < 8; ++r) B[lp(d + r * Ns)] = w[r];
    }
    cx* tmp = A;
    A = B;
    B = tmp;
  }
  // last stage, Ns = L / 8: butterfly b < Ns has k = b and writes b + r Ns
  __syncthreads();
  {
    const int sh = log2T - log2Ns - 3;
#pragma unroll
    for (int u = 0; u < NB8; ++u) {
      const int b = t + u * nts;
      cx w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = A[lp(b + r * eighth)];
      twiddle(w, b, sh);
      idft8(w);
#pragma unroll
      for (int r = 0; r < 8; ++r) v[u + r * NB8] = w[r];
    }
  }
  cur = A == b0 ? 1 : 0;
}

// RB consecutive rows r0..r0+RB-1 through one workgroup, RC of them at a
// time (RC = 1 or RB): the threads form RC slots of blockDim.x / RC threads,
// slot s owning LDS buf[s Lp ..) (Lp = padded_len(L)) and rows s, s + RC, ...
// Each row is read from HBM into registers one step ahead (while the previous
// one is transformed),
// multiplied by (-1)^(row+g) when pre_sign, transformed in LDS, and its
// cropped outputs times (-1)^q * drow[row] * dq[q'] are kept in registers.
// All RB rows of an output q' then leave as one RB-element segment at
// dst[q' out_stride_q + r0]: through LDS staged q'-major when RC = RB, or
// straight from registers when RC = 1 (one thread then holds all RB rows).
template <class real, int RB, int RC, int MAXQ, int PPT, bool DB>
__device__ __attribute__((always_inline)) inline void fft_rows_block(const typename CxF<real>::t* __restrict__ src, int64_t in_row_stride,
                                      typename CxF<real>::t* __restrict__ dst, int64_t out_stride_q, int L,
                                      int log2L, int ncrop, int crop_off, int r0, int pre_sign,
                                      const double* __restrict__ dq, const double* __restrict__ drow,
                                      typename CxF<real>::t* buf, const typename CxF<real>::t* __restrict__ tw,
                                      int log2T) {
  // twiddle tables behind the row buffers (RC, or 2 with db): lo (64
  // entries), hi (2^log2T / 64)
  typename CxF<real>::t* tw_lo = buf + (size_t)(DB ? 2 : RC) * padded_len(L);
  typename CxF<real>::t* tw_hi = tw_lo + 64;
  {
    const int ntw = 64 + max(1, (1 << log2T) >> 6);
    for (int i = threadIdx.x; i < ntw; i += blockDim.x) tw_lo[i] = tw[i];
  }
  static_assert(RC == 1 || RC == RB, "rows per workgroup run one at a time or all at once");
  using cx = typename CxF<real>::t;
  constexpr int NJ = RB / RC;
  const int nts = blockDim.x / RC;
  const int slot = RC == 1 ? 0 : (int)threadIdx.x / nts;
  const int t = (int)threadIdx.x - slot * nts;
  cx* sbuf = buf + (size_t)slot * padded_len(L);
  cx outv[NJ][MAXQ];
  cx nxt[PPT];
  {
    const cx* s0 = src + (int64_t)slot * in_row_stride;
#pragma unroll
    for (int u = 0; u < PPT; ++u)
      if (t + u * nts < L) nxt[u] = s0[t + u * nts];
  }
  if constexpr (RC == 1 && DB) {
    {
      // register path (the host sets db when L == PPT nts, the crop keeps
      // the middle half, crop_off = L / 4 = (PPT / 4) nts, and two row
      // buffers fit the LDS): the cropped output qp = t + kq nts is element
      // crop_off + qp = t + (PPT / 4 + kq) nts of the row, register
      // PPT / 4 + kq, an index fixed at compile time
      constexpr int U0 = PPT / 4;
      static_assert(U0 + MAXQ <= PPT || MAXQ > 4, "the cropped outputs are registers of the row");
      int cur = 0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int row = r0 + j;
        cx v[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          v[u] = nxt[u];
          if (pre_sign && ((row + t + u * nts) & 1)) {
            v[u].x = -v[u].x;
            v[u].y = -v[u].y;
          }
        }
        if (j + 1 < NJ) {
          const cx* s1 = src + (int64_t)(j + 1) * in_row_stride;
#pragma unroll
          for (int u = 0; u < PPT; ++u) nxt[u] = s1[t + u * nts];
        }
        reg_ifft_db<real, PPT>(v, buf, buf + padded_len(L), cur, L, log2L, t, nts, tw_lo, tw_hi, log2T);
        const double fr = drow ? drow[row] : 1.0;
#pragma unroll
        for (int kq = 0; kq < MAXQ; ++kq) {
          const int qp = t + kq * nts;
          if (U0 + kq < PPT && qp < ncrop) {
            const int q = qp + crop_off;
            double f = (q & 1) ? -fr : fr;
            if (dq) f *= dq[qp];
            const real fs = (real)f;
            cx w = v[U0 + kq < PPT ? U0 + kq : PPT - 1];
            w.x *= fs;
            w.y *= fs;
            outv[j][kq] = w;
          }
        }
      }
#pragma unroll
      for (int kq = 0; kq < MAXQ; ++kq) {
        const int qp = t + kq * nts;
        if (qp < ncrop) {
          cx* d = dst + (int64_t)qp * out_stride_q;
#pragma unroll
          for (int j = 0; j < RB; ++j) d[j] = outv[j][kq];
        }
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int rr = j * RC + slot;
    const int row = r0 + rr;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int g = t + u * nts;
      if (g < L) {
        cx v = nxt[u];
        if (pre_sign && ((row + g) & 1)) {
          v.x = -v.x;
          v.y = -v.y;
        }
        sbuf[lp(g)] = v;
      }
    }
    if (j + 1 < NJ) {
      const cx* s1 = src + (int64_t)(rr + RC) * in_row_stride;
#pragma unroll
      for (int u = 0; u < PPT; ++u)
        if (t + u * nts < L) nxt[u] = s1[t + u * nts];
    }
    __syncthreads();
    lds_ifft<real, PPT>(sbuf, L, log2L, t, nts, tw_lo, tw_hi, log2T);
    const double fr = drow ? drow[row] : 1.0;
#pragma unroll
    for (int kq = 0; kq < MAXQ; ++kq) {
      const int qp = t + kq * nts;
      if (qp < ncrop) {
        const int q = qp + crop_off;
        double f = (q & 1) ? -fr : fr;
        if (dq) f *= dq[qp];
        const real fs = (real)f;
        cx v = sbuf[lp(q)];
        v.x *= fs;
        v.y *= fs;
        outv[j][kq] = v;
      }
    }
    __syncthreads();
  }
  if constexpr (RC == 1) {
#pragma unroll
    for (int kq = 0; kq < MAXQ; ++kq) {
      const int qp = t + kq * nts;
      if (qp < ncrop) {
        cx* d = dst + (int64_t)qp * out_stride_q;
#pragma unroll
        for (int j = 0; j < RB; ++j) d[j] = outv[j][kq];
      }
    }
  } else {
    // RB * ncrop <= RB * L: the staging fits in the RC = RB row buffers
#pragma unroll
    for (int kq = 0; kq < MAXQ; ++kq) {
      const int qp = t + kq * nts;
      if (qp < ncrop) buf[qp * RB + slot] = outv[0][kq];
    }
    __syncthreads();
    const int tot = RB * ncrop;
    for (int e = threadIdx.x; e < tot; e += blockDim.x)
      dst[(int64_t)(e / RB) * out_stride_q + (e % RB)] = buf[e];
  }
}

template <class real, int RB, int RC, int MAXQ, int PPT, bool DB>
__global__ void k_fft_rows(const typename CxF<real>::t* __restrict__ in, int64_t in_row_stride,
                           typename CxF<real>::t* __restrict__ out, int64_t out_stride_q, int L, int log2L,
                           int ncrop, int crop_off, int rows, int pre_sign, const double* __restrict__ dq,
                           const double* __restrict__ drow, const typename CxF<real>::t* __restrict__ tw,
                           int log2T) {
  using cx = typename CxF<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* buf = reinterpret_cast<cx*>(smem_raw);
  const int r0 = (int)xcd_block(blockIdx.x, gridDim.x) * RB;
  fft_rows_block<real, RB, RC, MAXQ, PPT, DB>(in + (int64_t)r0 * in_row_stride, in_row_stride, out + r0,
                                              out_stride_q, L, log2L, ncrop, crop_off, r0, pre_sign, dq, drow, buf, tw,
                                              log2T);
}

// batched passes over the items of one grid size G (all with n = G / sigma),
// RB rows per workgroup: pass 1 maps row block b to item list[b*RB / G], grid
// rows b*RB % G ..; pass 2 maps it to item list[b*RB / n], intermediate rows
template <int RB, int RC, int MAXQ, int PPT, bool DB>
__global__ void k_fft_rows_batched(const BatchItem* __restrict__ items, const int* __restrict__ list,
                                   const BatchArgs* __restrict__ args, int pass, int L, int log2L, int n,
                                   const float2* __restrict__ tw, int log2T) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* buf = reinterpret_cast<float2*>(smem_raw);
  const int r = (int)xcd_block(blockIdx.x, gridDim.x) * RB;
  const int per = pass == 1 ? L : n;
  const BatchItem it = items[list[r / per]];
  const int row = r % per;
  const int crop_off = (L - n) / 2;
  if (pass == 1) {
    fft_rows_block<float, RB, RC, MAXQ, PPT, DB>(args->grid + it.grid_off + (int64_t)row * L, L,
                                             args->tmp + it.tmp_off + row, L, L, log2L, n, crop_off, row, 1, nullptr,
                                             nullptr, buf, tw, log2T);
  } else {
    const double* d = args->deapod + it.deapod_off;
    fft_rows_block<float, RB, RC, MAXQ, PPT, DB>(args->tmp + it.tmp_off + (int64_t)row * L, L,
                                             args->images + it.img_off + row, n, L, log2L, n, crop_off, row, 0, d,
                                             d, buf, tw, log2T);
  }
}

// launch shape of a row pass: PPT points per thread (8 while L / 8 threads fit
// a workgroup, else 16); nts = max(64, L / PPT) threads per row; MAXQ >= the
// cropped outputs per thread; RB rows per workgroup, as many as make each
// transposed store a 32-byte segment (4 float2 or 2 double2; 2 float2 at
// PPT 16, where 4 rows of outputs no longer fit in registers, and for rows
// of at most 2048 points, where 4 rows per workgroup leave too few
// workgroups to fill the chip: 1024-point rows 11 -> 10 us per pass), or 1
// when the row count is not a multiple of that; RC = RB rows at a time when RB row
// slots fit one workgroup (RB * nts <= 1024 threads, RB * L elements in 64 KiB
// of LDS, so two workgroups share a CU), else RC = 1
struct FftShape {
  int nts, ppt, maxq, rb, rc;
};

static FftShape fft_shape(int64_t L, int64_t ncrop, int64_t rows, int elem_bytes) {
  FftShape f;
  f.ppt = L <= 8192 ? 8 : 16;
  f.nts = (int)std::max<int64_t>(64, L / f.ppt);
  const int64_t q = (ncrop + f.nts - 1) / f.nts;
  f.maxq = q <= 4 && f.ppt == 8 ? 4 : 8;
  f.rb = (elem_bytes == 8 && f.ppt == 8) ? (L <= 2048 ? 2 : 4) : 2;
  if (rows % f.rb != 0) f.rb = 1;
  f.rc = (f.rb * f.nts <= 1024 && f.rb * padded_len((int)L) * elem_bytes <= 72 * 1024) ? f.rb : 1;
  return f;
}

// the register path of fft_rows_block (first and last stage in registers,
// two LDS row buffers): one-row-at-a-time shapes whose threads hold the whole
// row (L == PPT nts), the middle half cropped (oversampling 2: the cropped
// outputs are registers PPT / 4 .. of each thread), and two padded rows plus
// the twiddle tables within the 160 KiB of LDS
static int fft_db(const FftShape& f, int64_t L, int64_t crop_off, int elem_bytes) {
  if (f.rc != 1 || (int64_t)f.nts * f.ppt != L || crop_off * 4 != L) return 0;
  if (f.ppt / 4 + f.maxq > f.ppt) return 0;
  const int64_t lds = (2 * (int64_t)padded_len((int)L) + 64 + std::max<int64_t>(1, L >> 6)) * elem_bytes;
  return lds <= 160 * 1024 ? 1 : 0;
}

// calls fn.template operator()<RB, RC, MAXQ, PPT>() for the shape f
template <class Fn>
static void dispatch_shape(const FftShape& f, Fn&& fn) {
  const int mq = f.maxq == 4 ? 0 : (f.ppt == 8 ? 1 : 2);
  const int code = f.rb * 100 + f.rc * 10 + mq;
  switch (code) {
    case 440: fn.template operator()<4, 4, 4, 8>(); break;
    case 441: fn.template operator()<4, 4, 8, 8>(); break;
    case 410: fn.template operator()<4, 1, 4, 8>(); break;
    case 411: fn.template operator()<4, 1, 8, 8>(); break;
    case 220: fn.template operator()<2, 2, 4, 8>(); break;
    case 221: fn.template operator()<2, 2, 8, 8>(); break;
    case 210: fn.template operator()<2, 1, 4, 8>(); break;
    case 211: fn.template operator()<2, 1, 8, 8>(); break;
    case 212: fn.template operator()<2, 1, 8, 16>(); break;
    case 110: fn.template operator()<1, 1, 4, 8>(); break;
    case 111: fn.template operator()<1, 1, 8, 8>(); break;
    case 112: fn.template operator()<1, 1, 8, 16>(); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
}

struct BatchedLaunch {
  ftcg_batch_s* b;
  const int* list;
  int pass, rows;
  FftShape f;
  int L, log2L, n;
  const float2* tw;
  template <int RB, int RC, int MAXQ, int PPT, bool DB>
  void go() const {
    static bool attr_done = false;
    if (!attr_done) {
      FTCG_HIP(hipFuncSetAttribute((const void*)k_fft_rows_batched<RB, RC, MAXQ, PPT, DB>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      attr_done = true;
    }
    const size_t lds = ((size_t)(DB ? 2 : RC) * padded_len(L) + 64 + std::max(1, L >> 6)) * sizeof(float2);
    hipLaunchKernelGGL((k_fft_rows_batched<RB, RC, MAXQ, PPT, DB>), dim3((unsigned)(rows / RB)), dim3(f.nts * RC),
                       lds, b->stream, b->items_dev.as<BatchItem>(), list, b->args_dev.as<BatchArgs>(), pass, L, log2L,
                       n, tw, log2L);
  }
  template <int RB, int RC, int MAXQ, int PPT>
  void operator()() const {
    if (fft_db(f, L, (L - n) / 2, (int)sizeof(float2)))
      go<RB, RC, MAXQ, PPT, true>();
    else
      go<RB, RC, MAXQ, PPT, false>();
  }
};

void batch_fft_prepare() {}

void batch_fft(ftcg_batch_s* b) {
  const int* lists = b->group_items.as<int>();
  int64_t list_off = 0;
  size_t gi = 0;
  for (const auto& grp : b->fft_groups) {
    const float2* tw = b->twiddle.as<float2>() + b->twiddle_off[gi++];
    const int64_t G = b->items[grp[0]].G;
    const int n = b->items[grp[0]].n;
    int log2L = 0;
    while ((int64_t(1) << log2L) < G) ++log2L;
    const int* list = lists + list_off;
    for (int pass = 1; pass <= 2; ++pass) {
      const int per = pass == 1 ? (int)G : n;
      // row blocks must not straddle items: RB divides the rows of one item
      const FftShape f = fft_shape(G, n, per, (int)sizeof(float2));
      const int rows = (int)grp.size() * per;
      dispatch_shape(f, BatchedLaunch{b, list, pass, rows, f, (int)G, log2L, n, tw});
    }
    list_off += (int64_t)grp.size();
  }
  FTCG_HIP(hipGetLastError());
}

// sizes, stream and tables of one grid-to-image transform (from a plan, or
// from the allocation-free entry point's static scratch)
struct FftCtx {
  int dim;
  int64_t n, G;
  hipStream_t stream;
  const void* tw;        // two-level twiddle tables of the G-th roots of unity
  const double* deapod;  // n float64 factors 1 / Phi(x_p / sigma)
  void* tmp;             // n x G intermediate (2D)
  ftcg_plan timed;       // plan whose step timing records the passes (may be null)
};

template <class real>
struct RowsLaunch {
  const FftCtx* c;
  const void* in;
  int64_t in_row_stride;
  void* out;
  int64_t out_stride_q;
  int rows, pre_sign;
  FftShape f;
  const double* dq;
  const double* drow;
  template <int RB, int RC, int MAXQ, int PPT, bool DB>
  void go() const {
    using cx = typename CxF<real>::t;
    const int L = (int)c->G;
    int log2L = 0;
    while ((1 << log2L) < L) ++log2L;
    const int ncrop = (int)c->n;
    const int crop_off = (int)((c->G - c->n) / 2);
    const size_t lds = ((size_t)(DB ? 2 : RC) * padded_len(L) + 64 + std::max(1, L >> 6)) * sizeof(cx);
    static bool attr_done = false;
    if (!attr_done) {
      FTCG_HIP(hipFuncSetAttribute((const void*)k_fft_rows<real, RB, RC, MAXQ, PPT, DB>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      attr_done = true;
    }
    hipLaunchKernelGGL((k_fft_rows<real, RB, RC, MAXQ, PPT, DB>), dim3((unsigned)(rows / RB)), dim3(f.nts * RC), lds,
                       c->stream, static_cast<const cx*>(in), in_row_stride, static_cast<cx*>(out), out_stride_q, L,
                       log2L, ncrop, crop_off, rows, pre_sign, dq, drow, static_cast<const cx*>(c->tw), log2L);
    FTCG_HIP(hipGetLastError());
  }
  template <int RB, int RC, int MAXQ, int PPT>
  void operator()() const {
    if (fft_db(f, c->G, (c->G - c->n) / 2, (int)sizeof(typename CxF<real>::t)))
      go<RB, RC, MAXQ, PPT, true>();
    else
      go<RB, RC, MAXQ, PPT, false>();
  }
};

template <class real>
static void launch_rows(const FftCtx& c, const void* in, int64_t in_row_stride, void* out, int64_t out_stride_q,
                        int rows, int pre_sign, const double* dq, const double* drow) {
  const FftShape f = fft_shape(c.G, c.n, rows, (int)sizeof(typename CxF<real>::t));
  dispatch_shape(f, RowsLaunch<real>{&c, in, in_row_stride, out, out_stride_q, rows, pre_sign, f, dq, drow});
}

template <class real>
static void grid_to_image_t(const FftCtx& c, const void* grid, void* image) {
  const double* d = c.deapod;
  const int64_t G = c.G, n = c.n;
  ftcg_plan tp = c.timed;
  if (c.dim == 1) {
    if (tp) timing_begin(tp, STEP_FFT2);
    launch_rows<real>(c, grid, G, image, 1, 1, 1, d, nullptr);
    if (tp) timing_end(tp, STEP_FFT2);
    return;
  }
  if (tp) timing_begin(tp, STEP_FFT1);
  launch_rows<real>(c, grid, G, c.tmp, G, (int)G, 1, nullptr, nullptr);
  if (tp) timing_end(tp, STEP_FFT1);
  if (tp) timing_begin(tp, STEP_FFT2);
  launch_rows<real>(c, c.tmp, G, image, n, (int)n, 0, d, d);
  if (tp) timing_end(tp, STEP_FFT2);
}

void grid_to_image_raw(int dim, int64_t n, int64_t G, bool f64, hipStream_t stream, const void* tw,
                       const double* deapod, void* tmp, const void* grid, void* image) {
  const FftCtx c{dim, n, G, stream, tw, deapod, tmp, nullptr};
  if (f64)
    grid_to_image_t<double>(c, grid, image);
  else
    grid_to_image_t<float>(c, grid, image);
}

void grid_to_image(ftcg_plan p, const void* grid, void* image) {
  const FftCtx c{p->dim, p->n, p->G, p->stream, p->twiddle.p, p->deapod.as<double>(), p->fft_tmp.p, p};
  if (p->dtype == FTCG_F64)
    grid_to_image_t<double>(c, grid, image);
  else
    grid_to_image_t<float>(c, grid, image);
}

// deapodization factors 1 / Phi(x_p / sigma), Phi(t) = sqrt(pi/beta) exp(-pi^2 t^2 / beta), float64
__global__ void k_deapod(double* d, int64_t n, double sigma, double beta) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double pi = 3.141592653589793238462643383279502884;
  const double t = ((double)p - (double)(n / 2)) / (double)n / sigma;
  d[p] = 1.0 / (sqrt(pi / beta) * exp(-pi * pi * t * t / beta));
}

// two-level twiddle tables for w(j) = e^{2 pi i j / L}: tw[t] = w(t) for
// t < 64, then tw[64 + t] = w(64 t) for t < max(1, L / 64); float64, rounded once
template <class cx>
__global__ void k_twiddles(cx* tw, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nhi = L >= 64 ? L / 64 : 1;
  if (i >= 64 + nhi) return;
  const double j = i < 64 ? (double)i : 64.0 * (double)(i - 64);
  double s, c;
  sincospi(2.0 * j / (double)L, &s, &c);
  tw[i].x = c;
  tw[i].y = s;
}

int64_t twiddle_entries(int64_t L) { return 64 + (L >= 64 ? L / 64 : 1); }

void compute_twiddles(void* tw, int64_t L, bool f64, hipStream_t s) {
  const unsigned nb = (unsigned)((twiddle_entries(L) + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(k_twiddles<double2>, dim3(nb), dim3(256), 0, s, static_cast<double2*>(tw), (int)L);
  else
    hipLaunchKernelGGL(k_twiddles<float2>, dim3(nb), dim3(256), 0, s, static_cast<float2*>(tw), (int)L);
  FTCG_HIP(hipGetLastError());
}

void compute_deapod_raw(double* d, int64_t n, double sigma, double beta, hipStream_t s) {
  hipLaunchKernelGGL(k_deapod, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n, sigma, beta);
  FTCG_HIP(hipGetLastError());
}

void compute_deapod(ftcg_plan p) { compute_deapod_raw(p->deapod.as<double>(), p->n, p->sigma, p->beta, p->stream); }

}  // namespace ftcg

namespace ftcg {

// ---------------------------------------------------------------------------
// Forward transform passes (the adjoint of the passes above), for the
// type-2 transform: H[g] = sum_q J[q] e^{-2 pi i (g - G/2)(q - G/2)/G} over
// the centred window J[q] = image[q - (G - n)/2] (zero elsewhere). As above,
// with G divisible by 4 this is (-1)^g sum_q (-1)^q J[q] e^{-2 pi i g q / G},
// and the forward DFT is the conjugate of the inverse DFT of the conjugate,
// so each transform runs through the same in-LDS inverse FFT.
//
// These passes write every one of the G outputs of a transform (twice the
// data they read), so they read strided and write contiguous: a workgroup
// takes RB consecutive columns of its input (the n positions p of column r at
// in[p in_stride + r], read as RB-element, 32-byte segments), forms for each
// column the zero row of length G with the n values at offset (G - n)/2,
// times dq[p] drow[r] (-1)^q and conjugated, transforms it, and writes its G
// outputs, conjugated and times (-1)^g, as one contiguous row
// out[r out_row_stride + g]:
//   pass A: columns p1 of the image I[p0][p1]   -> T[p1][g0]  (n x G)
//   pass B: columns g0 of T (positions p1)      -> H[g0][g1]  (G x G), the
//           grid's own layout.
// ---------------------------------------------------------------------------
template <class real, int PPT, int RB>
__global__ void k_fft_cols_fwd(const typename CxF<real>::t* __restrict__ in, int64_t in_stride,
                               typename CxF<real>::t* __restrict__ out, int64_t out_row_stride, int L, int log2L,
                               int n, int crop_off, const double* __restrict__ dq, const double* __restrict__ drow,
                               const typename CxF<real>::t* __restrict__ tw, int log2T) {
  using cx = typename CxF<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* buf = reinterpret_cast<cx*>(smem_raw);
  cx* tw_lo = buf + padded_len(L);
  cx* tw_hi = tw_lo + 64;
  const int ntw = 64 + max(1, (1 << log2T) >> 6);
  for (int i = threadIdx.x; i < ntw; i += blockDim.x) tw_lo[i] = tw[i];
  const int nts = blockDim.x, t = threadIdx.x;
  const int r0 = (int)xcd_block(blockIdx.x, gridDim.x) * RB;
  double fc[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) fc[j] = drow ? drow[r0 + j] : 1.0;
  // this thread's positions of all RB columns, scaled and conjugated: the
  // first column straight into the LDS row, the others held in registers
  cx x[PPT][RB > 1 ? RB - 1 : 1];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int g = t + u * nts;
    const int p = g - crop_off;
    cx v0;
    v0.x = (real)0;
    v0.y = (real)0;
#pragma unroll
    for (int j = 1; j < RB; ++j) x[u][j - 1] = v0;
    if (g < L && p >= 0 && p < n) {
      const cx* src = in + (int64_t)p * in_stride + r0;
      double f = (g & 1) ? -1.0 : 1.0;
      if (dq) f *= dq[p];
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const cx v = src[j];
        const real fs = (real)(f * fc[j]);
        cx w;
        w.x = v.x * fs;
        w.y = -v.y * fs;   // conjugate
        if (j == 0)
          v0 = w;
        else
          x[u][j - 1] = w;
      }
    }
    if (g < L) buf[lp(g)] = v0;
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    if (j > 0) {
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int g = t + u * nts;
        if (g < L) buf[lp(g)] = x[u][j - 1];
      }
    }
    __syncthreads();
    lds_ifft<real, PPT>(buf, L, log2L, t, nts, tw_lo, tw_hi, log2T);
    cx* dst = out + (int64_t)(r0 + j) * out_row_stride;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int g = t + u * nts;
      if (g < L) {
        cx v = buf[lp(g)];
        const real sg = (g & 1) ? (real)-1 : (real)1;
        v.x *= sg;
        v.y *= -sg;     // conjugate
        dst[g] = v;
      }
    }
    __syncthreads();
  }
}

template <class real, int PPT, int RB>
static void launch_fwd_cols(const void* in, int64_t in_stride, void* out, int64_t out_row_stride, int64_t L,
                            int64_t n, int cols, const double* dq, const double* drow, const void* tw,
                            hipStream_t s) {
  using cx = typename CxF<real>::t;
  int log2L = 0;
  while ((int64_t(1) << log2L) < L) ++log2L;
  const int nts = (int)std::max<int64_t>(64, L / PPT);
  const size_t lds = ((size_t)padded_len((int)L) + 64 + std::max<int64_t>(1, L >> 6)) * sizeof(cx);
  static bool attr_done = false;
  if (!attr_done) {
    FTCG_HIP(hipFuncSetAttribute((const void*)k_fft_cols_fwd<real, PPT, RB>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_done = true;
  }
  hipLaunchKernelGGL((k_fft_cols_fwd<real, PPT, RB>), dim3((unsigned)(cols / RB)), dim3(nts), lds, s,
                     static_cast<const cx*>(in), in_stride, static_cast<cx*>(out), out_row_stride, (int)L, log2L,
                     (int)n, (int)((L - n) / 2), dq, drow, static_cast<const cx*>(tw), log2L);
  FTCG_HIP(hipGetLastError());
}

// RB columns per workgroup: 4 in float32 (32-byte read segments; the inputs
// of the other three columns held in registers bring the kernel to the 128
// VGPRs per lane of 1024-thread workgroups, with 2 spilled), else 1 (two
// float64 columns spill 20 VGPRs; float32 rows of 16384 points take 16
// points per thread)
template <class real, int PPT>
static void fwd_cols_rb(const void* in, int64_t in_stride, void* out, int64_t out_row_stride, int64_t L, int64_t n,
                        int cols, const double* dq, const double* drow, const void* tw, hipStream_t s) {
  constexpr int RB = (PPT == 8 && sizeof(real) == 4) ? 4 : 1;
  if (cols % RB == 0)
    launch_fwd_cols<real, PPT, RB>(in, in_stride, out, out_row_stride, L, n, cols, dq, drow, tw, s);
  else
    launch_fwd_cols<real, PPT, 1>(in, in_stride, out, out_row_stride, L, n, cols, dq, drow, tw, s);
}

// columns of n positions (column r at in[p in_stride + r]) -> zero-padded
// length-G forward DFTs with the centred sign convention, one contiguous row
// of out per column
void fft_cols_forward(bool f64, const void* in, int64_t in_stride, void* out, int64_t out_row_stride, int64_t G,
                      int64_t n, int cols, const double* dq, const double* drow, const void* tw, hipStream_t s) {
  if (f64) {
    if (G <= 8192)
      fwd_cols_rb<double, 8>(in, in_stride, out, out_row_stride, G, n, cols, dq, drow, tw, s);
    else
      throw StatusError{FTCG_EUNSUPPORTED};
  } else {
    if (G <= 8192)
      fwd_cols_rb<float, 8>(in, in_stride, out, out_row_stride, G, n, cols, dq, drow, tw, s);
    else
      fwd_cols_rb<float, 16>(in, in_stride, out, out_row_stride, G, n, cols, dq, drow, tw, s);
  }
}

}  // namespace ftcg
