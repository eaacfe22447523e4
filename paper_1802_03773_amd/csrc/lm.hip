// Levenberg-Marquardt iteration kernels (Backtrack LM of QRkit Section 5.2, Nielsen's
// gain-ratio damping rule) for the synthetic model f(x) = J0 phi(x) - y with the elementwise
// phi(t) = t + c t^3, whose Jacobian J(x) = J0 diag(phi'(x)) keeps the pattern of J0.
// Every kernel serves a batch of independent problems; all state (x, lambda, nu, costs) is
// on the device, so one iteration can be captured into a graph and replayed.
//
// Per iteration, per problem:
//   eval at x      : J(x) (stored), b = -f(x) (stored), d = column norms of J(x) (1 for a zero
//                    column), J^T f, F = |f|^2 / 2
//   factor + solve : p from the structured QR (libqrkit's factor and solve kernels)
//   pred           : 1/2 p^T (lam D^2 p - J^T f)         (= L(0) - L(p), L(h) = |f + J h|^2 / 2)
//   eval at x + p  : F_new = |f(x + p)|^2 / 2
//   accept         : rho = (F - F_new) / pred; rho > 0: x += p, lam *= max(1/3, 1 - (2 rho - 1)^3),
//                    nu = 2; else lam *= nu, nu *= 2
// Sums are deterministic (fixed-order per wave, per workgroup and per problem).
#include <algorithm>
#include <type_traits>

#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_lm.hpp"

namespace qrk {

__device__ __forceinline__ double lm_phi(double t, double c) { return t + c * t * t * t; }
__device__ __forceinline__ double lm_dphi(double t, double c) { return 1.0 + 3.0 * c * t * t; }

// ---------------------------------------------------------------------------------------
// Block-angular model evaluation: workgroup w serves the packs of problem wg_prob[w] (the
// refinement's assignment), one wave per pack of whole blocks.  The pack's rows of B0 are read
// once, 16 rows at a time with coalesced loads (lane = column), and staged in the wave's LDS
// tile; each row's B0 phi(u_B) is summed from the tile by four lanes, and J's B rows and their
// column sums come from the registers the rows were loaded into.
// JAC: writes A = A0 diag(phi'(u_blk)), B = B0 diag(phi'(u_B)), b = -f, the block columns'
//      d and J^T f, and per-workgroup partials of sum_r B_rj^2, sum_r B_rj f_r and sum_r f_r^2.
// !JAC: only the partial of sum_r f_r^2, at u = x + p.
// sum_r f_r^2 is written per pack (fpart[pack]), in the same order in both passes whatever the
// waves per workgroup, so that F and F_new of the same point agree bit for bit.
// ---------------------------------------------------------------------------------------
template <typename T, bool JAC>
__global__ void __launch_bounds__(JAC ? 256 : 512)
k_lmba_eval(const ProbDesc* __restrict__ probs, const int32_t* __restrict__ wg_prob,
            const int64_t* __restrict__ pack_blk, int n, const int64_t* __restrict__ row_off,
            const T* __restrict__ A0, const T* __restrict__ B0, const T* __restrict__ y, double c,
            const double* __restrict__ x, const double* __restrict__ pstep, T* __restrict__ A,
            T* __restrict__ B, T* __restrict__ b, double* __restrict__ d, double* __restrict__ gJ,
            double* __restrict__ part, double* __restrict__ fpart) {
  constexpr int CH = 16;      // rows per staged chunk
  constexpr int LS = CH + 1;  // column stride of the staged tile
  // waves per workgroup: the residual-only pass keeps less per wave, so eight fit the LDS
  constexpr int WG = JAC ? 4 : 8;
  __shared__ T tile_all[WG][kMaxDense * LS];
  __shared__ double phB[kMaxDense], dphB[kMaxDense];
  __shared__ double rr[WG][64];
  __shared__ double av[JAC ? WG : 1][64][8];
  __shared__ int rowblk[WG][64];
  __shared__ double red2[JAC ? WG : 1][kMaxDense], redf[JAC ? WG : 1][kMaxDense];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int pi = wg_prob[blockIdx.x];
  const ProbDesc& P = probs[pi];
  const int nB = P.nB;
  const int64_t koff = P.koff, noff = P.noff, moff = P.moff, ldb = P.ldb;
  const int64_t offB = noff + P.K * n;
  const T* B0p = B0 + P.boff;
  T* Bp = B + P.boff;
  T* tile = tile_all[wv];
  for (int j = threadIdx.x; j < kMaxDense; j += blockDim.x) {
    double ph = 0.0, dph = 0.0;  // zero past nB: the staged tile is zero there too
    if (j < nB) {
      const double u = x[offB + j] + (JAC ? 0.0 : pstep[offB + j]);
      ph = lm_phi(u, c);
      dph = lm_dphi(u, c);
    }
    phB[j] = ph;
    dphB[j] = dph;
  }
  __syncthreads();
  double s2a = 0.0, s2b = 0.0, sfa = 0.0, sfb = 0.0;  // columns lane, lane + 64
  double fsq = 0.0;
  const int qi = lane & 15, qq = lane >> 4;  // row pass: row qi of the chunk, columns 4t + qq
  const bool c0ok = lane < nB, c1ok = lane + 64 < nB;
  const int64_t lw = blockIdx.x - P.wg0;
  const int64_t pend = P.pack0 + P.npacks;
  for (int64_t pk = P.pack0 + lw * WG + wv; pk < pend; pk += (int64_t)P.nwg * WG) {
    const int64_t b0 = pack_blk[pk];
    const int nb = (int)(pack_blk[pk + 1] - b0);
    const int64_t pr0 = row_off[b0];
    const int prows = (int)(row_off[b0 + nb] - pr0);
    if (lane < nb) {
      const int lo = (int)(row_off[b0 + lane] - pr0), hi = (int)(row_off[b0 + lane + 1] - pr0);
      for (int r = lo; r < hi; ++r) rowblk[wv][r] = lane;
    }
    wave_lds_sync();
    for (int c0 = 0; c0 < prows; c0 += CH) {
      const int last = prows - 1 - c0;  // rows past the pack re-read its last row and are skipped
      // stage the chunk's rows of B0, coalesced across lanes (lane = column)
      T v0[CH], v1[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int ri = i < last ? i : last;
        const int64_t roff = (pr0 + c0 + ri - moff) * ldb;
        v0[i] = c0ok ? B0p[roff + lane] : T(0);
        v1[i] = c1ok ? B0p[roff + lane + 64] : T(0);
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        tile[lane * LS + i] = v0[i];
        tile[(lane + 64) * LS + i] = v1[i];
      }
      wave_lds_sync();
      // B0 phi(u_B) for row c0 + qi: lanes qi, qi + 16, qi + 32, qi + 48 split the columns
      double acc = 0.0;
      auto tier = [&](auto t_begin) {
        constexpr int tb = decltype(t_begin)::value;
#pragma unroll
        for (int t = tb; t < tb + 8; ++t) acc += (double)tile[(4 * t + qq) * LS + qi] * phB[4 * t + qq];
      };
      tier(std::integral_constant<int, 0>{});
      if (nB > 32) tier(std::integral_constant<int, 8>{});
      if (nB > 64) tier(std::integral_constant<int, 16>{});
      if (nB > 96) tier(std::integral_constant<int, 24>{});
      acc += __shfl_xor(acc, 16, 64);
      acc += __shfl_xor(acc, 32, 64);
      if (qq == 0 && qi <= last) {
        const int r = c0 + qi;
        const int64_t row = pr0 + r;
        const int64_t lb = b0 - koff + rowblk[wv][r];
        double f = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (k < n) {
            const double u = x[noff + lb * n + k] + (JAC ? 0.0 : pstep[noff + lb * n + k]);
            const double a0 = (double)A0[row * n + k];
            f += a0 * lm_phi(u, c);
            if constexpr (JAC) {
              const T a = (T)(a0 * lm_dphi(u, c));
              A[row * n + k] = a;
              av[wv][r][k] = (double)a;
            }
          }
        }
        f += acc - (double)y[row];
        rr[wv][r] = f;
        fsq += f * f;  // lane qi: rows qi, qi + 16, ... of this pack, in order
        if (JAC) b[row] = (T)(-f);
      }
      wave_lds_sync();
      if (JAC) {
        // J's B rows from the staged registers: scale, store (coalesced), column sums
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          if (i <= last) {
            const int64_t roff = (pr0 + c0 + i - moff) * ldb;
            const double fr = rr[wv][c0 + i];
            if (c0ok) {
              const T v = (T)((double)v0[i] * dphB[lane]);
              Bp[roff + lane] = v;
              s2a += (double)v * (double)v;
              sfa += (double)v * fr;
            }
            if (c1ok) {
              const T v = (T)((double)v1[i] * dphB[lane + 64]);
              Bp[roff + lane + 64] = v;
              s2b += (double)v * (double)v;
              sfb += (double)v * fr;
            }
          }
        }
      }
      wave_lds_sync();  // the next chunk overwrites the tile
    }
    if constexpr (JAC) {
      // block columns: lane per block
      if (lane < nb) {
        const int64_t lb = b0 - koff + lane;
        const int lo = (int)(row_off[b0 + lane] - pr0), hi = (int)(row_off[b0 + lane + 1] - pr0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (k < n) {
            double sq = 0.0, gf = 0.0;
            for (int r = lo; r < hi; ++r) {
              const double a = av[wv][r][k];
              sq += a * a;
              gf += a * rr[wv][r];
            }
            d[noff + lb * n + k] = sq > 0.0 ? sqrt(sq) : 1.0;
            gJ[noff + lb * n + k] = gf;
          }
        }
      }
    }
    // the pack's sum of f^2: butterfly across the wave (every lane ends with the same bits)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) fsq += __shfl_xor(fsq, off, 64);
    if (lane == 0) fpart[pk] = fsq;
    fsq = 0.0;
    wave_lds_sync();
  }
  // fixed-order reduction of the column sums: the workgroup's waves in order
  if constexpr (JAC) {
    red2[wv][lane] = s2a;
    red2[wv][lane + 64] = s2b;
    redf[wv][lane] = sfa;
    redf[wv][lane + 64] = sfb;
  }
  __syncthreads();
  if constexpr (JAC) {
    double* pw = part + (int64_t)blockIdx.x * 2 * kMaxDense;
    for (int j = threadIdx.x; j < nB; j += blockDim.x) {
      double a2 = red2[0][j], af = redf[0][j];
#pragma unroll
      for (int w = 1; w < WG; ++w) {
        a2 += red2[w][j];
        af += redf[w][j];
      }
      pw[j] = a2;
      pw[kMaxDense + j] = af;
    }
  }
}

// Per problem (one workgroup each): the dense columns' d and J^T f from the workgroup
// partials (JAC), and F = sum f^2 / 2 into Fout[p] from the per-pack partials.
template <bool JAC>
__global__ void __launch_bounds__(1024)
k_lmba_reduce(const ProbDesc* __restrict__ probs, int n, const double* __restrict__ part,
              const double* __restrict__ fpart, double* __restrict__ d, double* __restrict__ gJ,
              double* __restrict__ Fout) {
  // Fixed-order two-level sums over the problem's workgroup partials: thread (seg, j) sums
  // segment seg of the partials of column j (eight loads in flight), then the eight segments are
  // added in order; the F partials go through a 1,024-wide tree.
  constexpr int SEG = 8;
  __shared__ double s2_all[SEG][kMaxDense];
  __shared__ double sf_all[SEG][kMaxDense];
  __shared__ double red[1024];
  const int pi = blockIdx.x;
  const ProbDesc& P = probs[pi];
  const int t = threadIdx.x;
  const int seg = t / kMaxDense, j = t % kMaxDense;
  const int64_t offB = P.noff + P.K * n;
  const int64_t w0 = P.wg0, nw = P.nwg;
  if (JAC) {
    const int64_t per = (nw + SEG - 1) / SEG;
    const int64_t lo = w0 + seg * per, hi = w0 + (seg + 1) * per < w0 + nw ? w0 + (seg + 1) * per : w0 + nw;
    double s2 = 0.0, sf = 0.0;
    if (j < P.nB) {
      for (int64_t w = lo; w < hi; w += 8) {
        double a2[8], af[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const bool ok = w + u < hi;
          a2[u] = ok ? part[(w + u) * 2 * kMaxDense + j] : 0.0;
          af[u] = ok ? part[(w + u) * 2 * kMaxDense + kMaxDense + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          s2 += a2[u];
          sf += af[u];
        }
      }
    }
    s2_all[seg][j] = s2;
    sf_all[seg][j] = sf;
  }
  double fs = 0.0;
  for (int64_t k = P.pack0 + t; k < P.pack0 + P.npacks; k += 1024) fs += fpart[k];
  red[t] = fs;
  __syncthreads();
  if (JAC && seg == 0 && j < P.nB) {
    double s2 = 0.0, sf = 0.0;
#pragma unroll
    for (int g = 0; g < SEG; ++g) {
      s2 += s2_all[g][j];
      sf += sf_all[g][j];
    }
    d[offB + j] = s2 > 0.0 ? sqrt(s2) : 1.0;
    gJ[offB + j] = sf;
  }
  for (int h = 512; h >= 1; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) Fout[pi] = 0.5 * red[0];
}

// ---------------------------------------------------------------------------------------
// Banded model evaluation (P problems of M rows, N unknowns, w values per row starting at the
// nondecreasing column row_start[i]).  Rows: one thread per row, grid (ceil(M/256), P);
// JAC writes J(x) = vals0 diag(phi'(x)), b = -f and f, at x; !JAC evaluates at x + p.  Both
// write per-workgroup partials of sum f^2.  Columns: one thread per column, summing over the
// rows that cover it (found by binary search on row_start) in row order.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t lm_row_start(const int32_t* rs, int64_t i, int64_t N, int w) {
  int64_t s = rs[i];
  return s < 0 ? 0 : (s > N - w ? N - w : s);
}

template <typename T, bool JAC>
__global__ void __launch_bounds__(256)
k_lmbd_rows(int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start, const T* __restrict__ vals0,
            const T* __restrict__ y, double c, const double* __restrict__ x, const double* __restrict__ pstep,
            T* __restrict__ vals, T* __restrict__ b, double* __restrict__ f, double* __restrict__ fpart) {
  __shared__ double red[256];
  const int64_t prob = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double fi = 0.0;
  if (i < M) {
    const int64_t row = prob * M + i;
    const int64_t s = lm_row_start(row_start + prob * M, i, N, w);
    for (int k = 0; k < w; ++k) {
      const int64_t col = prob * N + s + k;
      const double u = x[col] + (JAC ? 0.0 : pstep[col]);
      const double v0 = (double)vals0[row * w + k];
      fi += v0 * lm_phi(u, c);
      if (JAC) vals[row * w + k] = (T)(v0 * lm_dphi(u, c));
    }
    fi -= (double)y[row];
    if (JAC) {
      b[row] = (T)(-fi);
      f[row] = fi;
    }
  }
  red[threadIdx.x] = fi * fi;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) fpart[prob * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_lmbd_fsum(int nblk, const double* __restrict__ fpart, double* __restrict__ Fout) {
  const int prob = blockIdx.x;
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += fpart[(int64_t)prob * nblk + k];
  Fout[prob] = 0.5 * s;
}

// The row kernel with the band width W (<= 15) at compile time: every load of a row is in
// flight at once.  Same arithmetic, in the same order, as k_lmbd_rows.
template <typename T, bool JAC, int W>
__global__ void __launch_bounds__(256)
k_lmbd_rows_w(int64_t M, int64_t N, const int32_t* __restrict__ row_start, const T* __restrict__ vals0,
              const T* __restrict__ y, double c, const double* __restrict__ x, const double* __restrict__ pstep,
              T* __restrict__ vals, T* __restrict__ b, double* __restrict__ f, double* __restrict__ fpart) {
  __shared__ double red[256];
  const int64_t prob = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double fi = 0.0;
  if (i < M) {
    const int64_t row = prob * M + i;
    const int64_t s = lm_row_start(row_start + prob * M, i, N, W);
    const double* xp = x + prob * N + s;
    const double* pp = JAC ? nullptr : pstep + prob * N + s;
    double u[W];
    T v0[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      u[k] = xp[k] + (JAC ? 0.0 : pp[k]);
      v0[k] = vals0[row * W + k];
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      fi += (double)v0[k] * lm_phi(u[k], c);
      if (JAC) vals[row * W + k] = (T)((double)v0[k] * lm_dphi(u[k], c));
    }
    fi -= (double)y[row];
    if (JAC) {
      b[row] = (T)(-fi);
      f[row] = fi;
    }
  }
  red[threadIdx.x] = fi * fi;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) fpart[prob * gridDim.x + blockIdx.x] = red[0];
}

// Column norms and J^T f with the first-row table fr [P][N+1] (first row whose start is >= c):
// a workgroup covers 256 consecutive columns of one problem and copies its rows' values, starts
// and residuals into LDS with coalesced loads; each column then sums its rows in row order
// (the order of k_lmbd_cols).  Ranges beyond the LDS capacity read their rows from memory.
template <typename T>
__global__ void __launch_bounds__(256)
k_lmbd_cols_t(int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start, const int32_t* __restrict__ fr,
              const T* __restrict__ vals, const double* __restrict__ f, double* __restrict__ d,
              double* __restrict__ gJ) {
  constexpr int CAP = 1024;
  constexpr int VCAP = 40960 / (int)sizeof(T);
  __shared__ int32_t s_st[CAP];
  __shared__ double s_f[CAP];
  __shared__ T s_v[VCAP];
  const int64_t prob = blockIdx.y;
  const int64_t c0 = (int64_t)blockIdx.x * 256;
  const int64_t j = c0 + threadIdx.x;
  const int32_t* rs = row_start + prob * M;
  const int32_t* fp = fr + prob * (N + 1);
  const double* fv = f + prob * M;
  const T* V = vals + prob * M * w;
  auto row_at = [&](int64_t cc) -> int64_t {
    cc = cc < 0 ? 0 : (cc > N ? N : cc);
    const int64_t r = fp[cc];
    return r < 0 ? 0 : (r > M ? M : r);
  };
  const int64_t lo = row_at(c0 - w + 1);
  int64_t hi = row_at(c0 + 256);
  hi = hi < lo ? lo : hi;
  const int64_t n = hi - lo;
  const bool staged = n <= CAP && n * w <= VCAP;
  if (staged) {
    const int64_t nv = n * w;
    const T* Vlo = V + lo * w;
    for (int64_t i0 = 0; i0 < nv; i0 += 256 * 8) {
      T buf[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        buf[u] = i < nv ? Vlo[i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        if (i < nv) s_v[i] = buf[u];
      }
    }
    for (int64_t i0 = 0; i0 < n; i0 += 256 * 4) {
      int32_t sb[4];
      double fb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        sb[u] = i < n ? (int32_t)lm_row_start(rs, lo + i, N, w) : 0;
        fb[u] = i < n ? fv[lo + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        if (i < n) {
          s_st[i] = sb[u];
          s_f[i] = fb[u];
        }
      }
    }
    __syncthreads();
  }
  if (j >= N) return;
  int64_t a = row_at(j - w + 1), e = row_at(j + 1);
  double sq = 0.0, gf = 0.0;
  if (staged) {
    a = a < lo ? lo : a;
    e = e > hi ? hi : e;
    const int i1 = (int)(e - lo);
    for (int i0 = (int)(a - lo); i0 < i1; i0 += 8) {
      int kk[8];
      double ff[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u < i1 ? i0 + u : i1 - 1;
        kk[u] = (int)(j - s_st[i]);
        ff[u] = s_f[i];
      }
      T vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u < i1 ? i0 + u : i1 - 1;
        const int k = kk[u] < 0 ? 0 : (kk[u] >= w ? w - 1 : kk[u]);
        vv[u] = s_v[i * w + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < i1 && kk[u] >= 0 && kk[u] < w) {
          const double v = (double)vv[u];
          sq += v * v;
          gf += v * ff[u];
        }
    }
  } else {
    for (int64_t i = a; i < e; ++i) {
      const int64_t k = j - lm_row_start(rs, i, N, w);
      if (k < 0 || k >= w) continue;
      const double v = (double)V[i * w + k];
      sq += v * v;
      gf += v * fv[i];
    }
  }
  d[prob * N + j] = sq > 0.0 ? sqrt(sq) : 1.0;
  gJ[prob * N + j] = gf;
}

// ---------------------------------------------------------------------------------------
// Problem-generic pieces (unknowns of problem p: [noff[p], noff[p+1])).
// ---------------------------------------------------------------------------------------
// pred = p^T (lam D^2 p - J^T f) / 2, deterministic two-level sum: workgroup (bx, p) sums its
// 2,048 unknowns of problem p (eight per thread, loads in flight together) through an LDS
// tree into part[p][bx]; one workgroup per problem then adds the parts in a fixed tree.
constexpr int kPredChunk = 2048;
__global__ void __launch_bounds__(256)
k_lm_pred_part(const int64_t* __restrict__ noff, const double* __restrict__ p, const double* __restrict__ d,
               const double* __restrict__ gJ, const double* __restrict__ lam, double* __restrict__ part) {
  __shared__ double red[256];
  const int pi = blockIdx.y;
  const int64_t a = noff[pi], e = noff[pi + 1];
  const int64_t j0 = a + (int64_t)blockIdx.x * kPredChunk + threadIdx.x;
  const double l = lam[pi];
  double pv[8], dv[8], gv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t j = j0 + u * 256;
    const bool ok = j < e;
    pv[u] = ok ? p[j] : 0.0;
    dv[u] = ok ? d[j] : 0.0;
    gv[u] = ok ? gJ[j] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) s += pv[u] * (l * dv[u] * dv[u] * pv[u] - gv[u]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)pi * gridDim.x + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
k_lm_pred_final(int nbx, const double* __restrict__ part, double* __restrict__ pred) {
  __shared__ double red[256];
  const int pi = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nbx; k += 256) s += part[(int64_t)pi * nbx + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) pred[pi] = 0.5 * red[0];
}

// One workgroup: gain ratio, damping update and accept flag of every problem, the iteration
// log ([iter][p] = F, F_new, lam after, accepted) and the iteration counter.
__global__ void __launch_bounds__(256)
k_lm_accept(int P, const double* __restrict__ F, const double* __restrict__ Fnew, const double* __restrict__ pred,
            double* __restrict__ lam, double* __restrict__ nu, int* __restrict__ acc, int* __restrict__ iter,
            double* __restrict__ log, int max_log) {
  const int it = *iter;
  for (int pi = threadIdx.x; pi < P; pi += blockDim.x) {
    const double f0 = F[pi], f1 = Fnew[pi], pr = pred[pi];
    double rho = -1.0;
    if (pr > 0.0 && is_finite(f1) && is_finite(pr)) rho = (f0 - f1) / pr;
    double l = lam[pi], v = nu[pi];
    const bool ok = rho > 0.0;
    if (ok) {
      const double t = 2.0 * rho - 1.0;
      l *= fmax(1.0 / 3.0, 1.0 - t * t * t);
      v = 2.0;
    } else {
      l *= v;
      v *= 2.0;
    }
    lam[pi] = l;
    nu[pi] = v;
    acc[pi] = ok ? 1 : 0;
    if (it < max_log) {
      double* r = log + ((int64_t)it * P + pi) * 4;
      r[0] = f0;
      r[1] = f1;
      r[2] = l;
      r[3] = ok ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *iter = it + 1;
}

// x += p for the problems whose step was accepted: one thread per unknown, grid (., P).
__global__ void __launch_bounds__(256)
k_lm_step(const int64_t* __restrict__ noff, const int* __restrict__ acc, const double* __restrict__ p,
          double* __restrict__ x) {
  const int pi = blockIdx.y;
  if (!acc[pi]) return;
  const int64_t j = noff[pi] + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < noff[pi + 1]) x[j] += p[j];
}

__global__ void k_lm_init(int P, double* __restrict__ nu, int* __restrict__ iter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) nu[i] = 2.0;
  if (i == 0) *iter = 0;
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_lmba_eval(const BatchView& bv, bool jac, const T* A0, const T* B0, const T* y, double c,
                            const double* x, const double* p, T* A, T* B, T* b, double* d, double* gJ,
                            double* part, double* fpart, double* Fout, hipStream_t st) {
  if (bv.max_L > kMaxDense || bv.n > 8) return hipErrorInvalidValue;
  if (jac)
    hipLaunchKernelGGL((k_lmba_eval<T, true>), dim3(bv.nwg), dim3(256), 0, st, bv.probs, bv.wg_prob, bv.pack_blk,
                       bv.n, bv.row_off, A0, B0, y, c, x, p, A, B, b, d, gJ, part, fpart);
  else
    hipLaunchKernelGGL((k_lmba_eval<T, false>), dim3(bv.nwg), dim3(512), 0, st, bv.probs, bv.wg_prob,
                       bv.pack_blk, bv.n, bv.row_off, A0, B0, y, c, x, p, A, B, b, d, gJ, part, fpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (jac)
    hipLaunchKernelGGL((k_lmba_reduce<true>), dim3(bv.P), dim3(1024), 0, st, bv.probs, bv.n, part, fpart, d, gJ,
                       Fout);
  else
    hipLaunchKernelGGL((k_lmba_reduce<false>), dim3(bv.P), dim3(1024), 0, st, bv.probs, bv.n, part, fpart, d, gJ,
                       Fout);
  return hipGetLastError();
}

int lm_pred_blocks(int64_t maxN) { return (int)std::max<int64_t>(1, (maxN + kPredChunk - 1) / kPredChunk); }

hipError_t launch_lm_control(int P, int64_t maxN, const int64_t* noff, const double* p, const double* d,
                             const double* gJ, double* lam, double* nu, const double* F, const double* Fnew,
                             double* pred, double* predpart, int* acc, int* iter, double* log, int max_log, double* x,
                             hipStream_t st, int stage) {
  if (stage == 0) {
    const int nbx = lm_pred_blocks(maxN);
    hipLaunchKernelGGL(k_lm_pred_part, dim3(nbx, P), dim3(256), 0, st, noff, p, d, gJ, lam, predpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lm_pred_final, dim3(P), dim3(256), 0, st, nbx, predpart, pred);
  } else {
    hipLaunchKernelGGL(k_lm_accept, dim3(1), dim3(256), 0, st, P, F, Fnew, pred, lam, nu, acc, iter, log, max_log);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nbx = (unsigned)std::max<int64_t>(1, (maxN + 255) / 256);
    hipLaunchKernelGGL(k_lm_step, dim3(nbx, P), dim3(256), 0, st, noff, acc, p, x);
  }
  return hipGetLastError();
}

hipError_t launch_lm_init(int P, double* nu, int* iter, hipStream_t st) {
  hipLaunchKernelGGL(k_lm_init, dim3((P + 255) / 256), dim3(256), 0, st, P, nu, iter);
  return hipGetLastError();
}


template <int A, int B, typename F>
inline void lm_host_for(F&& fn) {
  if constexpr (A < B) {
    fn(std::integral_constant<int, A>{});
    lm_host_for<A + 1, B>(fn);
  }
}

template <typename T>
hipError_t launch_lmbd_eval(int P, int64_t M, int64_t N, int w, bool jac, const int32_t* row_start, const int32_t* fr,
                            const T* vals0, const T* y, double c, const double* x, const double* p, T* vals, T* b,
                            double* f, double* d, double* gJ, double* fpart, double* Fout, hipStream_t st) {
  const int nblk = (int)((M + 255) / 256);
  if (P < 1 || nblk < 1) return hipErrorInvalidValue;
  dim3 grd(nblk, P);
  if (w <= 15) {
    lm_host_for<1, 16>([&](auto WW) {
      constexpr int W = decltype(WW)::value;
      if (w != W) return;
      if (jac)
        hipLaunchKernelGGL((k_lmbd_rows_w<T, true, W>), grd, dim3(256), 0, st, M, N, row_start, vals0, y, c, x, p,
                           vals, b, f, fpart);
      else
        hipLaunchKernelGGL((k_lmbd_rows_w<T, false, W>), grd, dim3(256), 0, st, M, N, row_start, vals0, y, c, x, p,
                           vals, b, f, fpart);
    });
  } else if (jac) {
    hipLaunchKernelGGL((k_lmbd_rows<T, true>), grd, dim3(256), 0, st, M, N, w, row_start, vals0, y, c, x, p, vals, b,
                       f, fpart);
  } else {
    hipLaunchKernelGGL((k_lmbd_rows<T, false>), grd, dim3(256), 0, st, M, N, w, row_start, vals0, y, c, x, p, vals,
                       b, f, fpart);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lmbd_fsum, dim3(P), dim3(64), 0, st, nblk, fpart, Fout);
  e = hipGetLastError();
  if (e != hipSuccess || !jac) return e;
  hipLaunchKernelGGL((k_lmbd_cols_t<T>), dim3((unsigned)((N + 255) / 256), P), dim3(256), 0, st, M, N, w, row_start,
                     fr, vals, f, d, gJ);
  return hipGetLastError();
}

#define QRK_INST(T)                                                                                      \
  template hipError_t launch_lmba_eval<T>(const BatchView&, bool, const T*, const T*, const T*, double,    \
                                          const double*, const double*, T*, T*, T*, double*, double*,      \
                                          double*, double*, double*, hipStream_t);                         \
  template hipError_t launch_lmbd_eval<T>(int, int64_t, int64_t, int, bool, const int32_t*, const int32_t*, const T*, const T*,  \
                                          double, const double*, const double*, T*, T*, double*, double*, double*, \
                                          double*, double*, hipStream_t);
QRK_INST(float)
QRK_INST(double)
#undef QRK_INST

}  // namespace qrk
