// Near-screen field and its transpose by the convolution theorem.
//
// Both near-field contractions are periodic convolutions over the element
// lattice whose kernel is the table of Section 3 (eq. sc, the Remark's
// order-p tables), with 8 moment channels on one side and the (p+1)^3 node
// channels on the other:
//
//   Psi_E[m] = sum_D sum_a T[a][D][m] C[E - D][a]    (element-to-point field)
//   B_E[a]   = sum_D sum_m T[a][D][m] g[E + D][m]    (its transpose, in the
//                                                     moment adjoint)
//
// With X^(k) = sum_E X[E] exp(-2 pi i k.E / n) and the table spectrum
//   S[k][a][m] = sum_D T[a][D][m] exp(-2 pi i k.D / n)
// they read Psi^_m(k) = sum_a S[k][a][m] C^_a(k) and
// B^_a(k) = sum_m conj(S[k][a][m]) g^_m(k) (T is real).  The same linear maps
// as the direct sums, evaluated with 3-D FFTs of the element lattice: about
// 2 * 8 * 216 * 16 FLOP per element for the products against 1.19 MFLOP per
// element for the direct sums; the work becomes memory-bound (the spectrum,
// 8 * 216 complex values per frequency, is read once per product).
//
// Layout: every transformed field is [config][z][y][x][channel] complex
// (double2), channel fastest, where two consecutive real channels form one
// complex channel: the moments C[E][8] are 4 complex channels in place, the
// node fields [E][216] are 108.  One complex FFT of the pair (X_2c + i X_2c+1)
// transforms both real channels; X^_2c(k) = (Z(k) + conj Z(-k)) / 2 and
// X^_2c+1(k) = (Z(k) - conj Z(-k)) / 2i separate them in the products, which
// also pack their two real outputs the same way, so the inverse transforms
// return real pairs directly.  The spectrum is kept for the half set of
// frequencies k_z in [0, n/2] (S(-k) = conj S(k)); each product handles the
// pair {k, -k} at once.
//
// FFTs: one kernel per axis, radix-2 decimation in time in LDS.  A block
// holds lb lines x cc channels of length n (at most 2048 complex values):
// rows of cc consecutive channels (and lb consecutive elements across the
// line for the y and z passes) are contiguous in memory.  Twiddles come from
// a table computed on the host.  n is a power of two, 8 .. 128.
#include "kernels.hpp"

namespace fep3m {

namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

constexpr int kFftCap = 2048;   // complex values per FFT block (32 KB of LDS)

// Frequency pair of half-set index kk: full indices of k and -k, and whether
// kk is the representative of its pair (the planes k_z = 0 and k_z = n/2
// hold both members; the lower (k_y, k_x) one is the representative).
__device__ __forceinline__ bool freq_pair(int kk, int n, int &fk, int &fm) {
  const int kx = kk % n, ky = (kk / n) % n, kz = kk / (n * n);
  const int mx = (n - kx) & (n - 1), my = (n - ky) & (n - 1), mz = (n - kz) & (n - 1);
  fk = (kz * n + ky) * n + kx;
  fm = (mz * n + my) * n + mx;
  if (kz == 0 || 2 * kz == n) return ky * n + kx <= my * n + mx;
  return true;
}

}  // namespace

// One axis of a batched 3-D FFT over [cfg][z][y][x][nch] complex values.
// EPI 0: store the transformed values to dst (src == dst allowed: a block
// reads all its values before it writes).  EPI 1 (last inverse pass of the
// field): the values are (Psi_2c, Psi_2c+1) of element E; store
// W_E[m] = phi(node of m) - Psi_m to Wout (float64 or float32), phi the
// order-po mesh potential.
template <bool INV, int EPI, class WT>
__global__ __launch_bounds__(256) void k_fft_axis(int n, int logn, int nch, int cc, int lb, int axis,
                                                  const double2 *src, double2 *dst, const double2 *__restrict__ tw,
                                                  const double *__restrict__ phi, WT *__restrict__ Wout, int po) {
  extern __shared__ double2 fsm[];
  const int U = lb * cc;
  double2 *buf = fsm;                 // [j][u], u = l cc + c
  double2 *tws = fsm + size_t(n) * U; // n / 2 twiddles
  const int nchunk = nch / cc, ng = n / lb;
  int b = blockIdx.x;
  const int chunk = b % nchunk;
  b /= nchunk;
  const int g = b % ng;
  b /= ng;
  const int outer = b % n;
  const int cfg = b / n;
  const size_t nc = size_t(nch);
  size_t sj, sl, so;
  if (axis == 0) { sj = nc; sl = size_t(n) * nc; so = size_t(n) * n * nc; }
  else if (axis == 1) { sj = size_t(n) * nc; sl = nc; so = size_t(n) * n * nc; }
  else { sj = size_t(n) * n * nc; sl = nc; so = size_t(n) * nc; }
  const size_t base = size_t(cfg) * n * n * n * nc + size_t(outer) * so + size_t(g) * lb * sl + size_t(chunk) * cc;
  const int tid = threadIdx.x, tot = n * U;
  for (int t = tid; t < n / 2; t += 256) tws[t] = tw[t];
  // load in bit-reversed order of j; the thread order follows memory
  for (int i = tid; i < tot; i += 256) {
    const int c = i % cc, r = i / cc;
    int j, l;
    if (axis == 0) { j = r % n; l = r / n; } else { l = r % lb; j = r / lb; }
    const int jr = int(__brev(unsigned(j)) >> (32 - logn));
    buf[jr * U + l * cc + c] = src[base + j * sj + l * sl + c];
  }
  __syncthreads();
  for (int s = 0; s < logn; ++s) {
    const int h = 1 << s;
    for (int t = tid; t < (n / 2) * U; t += 256) {
      const int u = t % U, bf = t / U;
      const int pos = bf & (h - 1);
      const int j0 = ((bf >> s) << (s + 1)) + pos, j1 = j0 + h;
      double2 w = tws[pos << (logn - 1 - s)];
      if (INV) w.y = -w.y;
      const double2 x0 = buf[j0 * U + u], x1 = cmul(buf[j1 * U + u], w);
      buf[j0 * U + u] = cadd(x0, x1);
      buf[j1 * U + u] = csub(x0, x1);
    }
    __syncthreads();
  }
  if (EPI == 0) {
    for (int i = tid; i < tot; i += 256) {
      const int c = i % cc, r = i / cc;
      int j, l;
      if (axis == 0) { j = r % n; l = r / n; } else { l = r % lb; j = r / lb; }
      dst[base + j * sj + l * sl + c] = buf[j * U + l * cc + c];
    }
  } else {
    const int Q1 = po + 1, NM = Q1 * Q1 * Q1, P = po * n;
    const size_t M = size_t(n) * n * n;
    phi += size_t(cfg) * P * P * P;
    for (int i = tid; i < tot; i += 256) {
      const int c = i % cc, r = i / cc;
      int j, l;
      if (axis == 0) { j = r % n; l = r / n; } else { l = r % lb; j = r / lb; }
      int ex, ey, ez;
      const int lc = g * lb + l;
      if (axis == 0) { ex = j; ey = lc; ez = outer; }
      else if (axis == 1) { ey = j; ex = lc; ez = outer; }
      else { ez = j; ex = lc; ey = outer; }
      const double2 v = buf[j * U + l * cc + c];
      const size_t E = size_t(cfg) * M + (size_t(ez) * n + ey) * n + ex;
      const int ch = chunk * cc + c;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = 2 * ch + q;
        const int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
        int gx = po * ex + mx, gy = po * ey + my, gz = po * ez + mz;
        gx -= gx >= P ? P : 0;
        gy -= gy >= P ? P : 0;
        gz -= gz >= P ? P : 0;
        const double ph = phi[(size_t(gz) * P + gy) * P + gx];
        Wout[E * NM + m] = WT(ph - (q == 0 ? v.x : v.y));
      }
    }
  }
}

// Forward product: Z_out(k) = (Psi^_2c(k) + i Psi^_2c+1(k)) * scale for the
// 108 channel pairs c (one lane each), at k and -k.
__global__ __launch_bounds__(128) void k_spec_psi(int n, int NF, int nm, const double2 *__restrict__ S,
                                                  const double2 *__restrict__ ZC, double2 *__restrict__ Zout,
                                                  double scale) {
  const int kk = blockIdx.x % NF, cfg = blockIdx.x / NF;
  int fk, fm;
  if (!freq_pair(kk, n, fk, fm)) return;
  const int c = threadIdx.x, nc = nm / 2;
  if (c >= nc) return;
  const size_t M = size_t(n) * n * n;
  ZC += size_t(cfg) * M * 4;
  Zout += size_t(cfg) * M * nc;
  double2 Ch[8];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double2 z = ZC[size_t(fk) * 4 + a], zm = ZC[size_t(fm) * 4 + a];
    Ch[2 * a] = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
    Ch[2 * a + 1] = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
  }
  const double2 *Sk = S + size_t(kk) * 8 * nm + 2 * c;
  double2 P0 = make_double2(0.0, 0.0), P1 = make_double2(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double2 s0 = Sk[a * nm], s1 = Sk[a * nm + 1];
    P0 = cadd(P0, cmul(s0, Ch[a]));
    P1 = cadd(P1, cmul(s1, Ch[a]));
  }
  Zout[size_t(fk) * nc + c] = make_double2((P0.x - P1.y) * scale, (P0.y + P1.x) * scale);
  if (fm != fk) Zout[size_t(fm) * nc + c] = make_double2((P0.x + P1.y) * scale, (P1.x - P0.y) * scale);
}

// Transposed product: B^_a(k) = sum_m conj(S[k][a][m]) g^_m(k); lanes take
// channel pairs, the 8 sums are reduced over the block in a fixed order.
__global__ __launch_bounds__(128) void k_spec_adj(int n, int NF, int nm, const double2 *__restrict__ S,
                                                  const double2 *__restrict__ Zg, double2 *__restrict__ ZA,
                                                  double scale) {
  __shared__ double red[2][16];
  const int kk = blockIdx.x % NF, cfg = blockIdx.x / NF;
  int fk, fm;
  if (!freq_pair(kk, n, fk, fm)) return;   // uniform over the block
  const int c = threadIdx.x, nc = nm / 2;
  const size_t M = size_t(n) * n * n;
  Zg += size_t(cfg) * M * nc;
  ZA += size_t(cfg) * M * 4;
  double acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
  if (c < nc) {
    const double2 z = Zg[size_t(fk) * nc + c], zm = Zg[size_t(fm) * nc + c];
    const double2 g0 = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
    const double2 g1 = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
    const double2 *Sk = S + size_t(kk) * 8 * nm + 2 * c;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double2 v = cadd(cmulc(Sk[a * nm], g0), cmulc(Sk[a * nm + 1], g1));
      acc[2 * a] = v.x;
      acc[2 * a + 1] = v.y;
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i)
    for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off, 64);
  const int w = c >> 6;
  if ((c & 63) == 0)
#pragma unroll
    for (int i = 0; i < 16; ++i) red[w][i] = acc[i];
  __syncthreads();
  if (c < 4) {
    const int j = c;
    const double2 A0 = make_double2(red[0][4 * j] + red[1][4 * j], red[0][4 * j + 1] + red[1][4 * j + 1]);
    const double2 A1 = make_double2(red[0][4 * j + 2] + red[1][4 * j + 2], red[0][4 * j + 3] + red[1][4 * j + 3]);
    ZA[size_t(fk) * 4 + j] = make_double2((A0.x - A1.y) * scale, (A0.y + A1.x) * scale);
    if (fm != fk) ZA[size_t(fm) * 4 + j] = make_double2((A0.x + A1.y) * scale, (A1.x - A0.y) * scale);
  }
}

// Table spectrum S[kk][a][m] over the half set of frequencies: 8 consecutive
// frequencies per block, one thread per node m, the phases
// exp(-2 pi i k.D / n) = tw[(k.D) mod n] of the block's frequencies in LDS.
template <int NSR>
__global__ __launch_bounds__(256) void k_spec_build(int n, int nm, const double *__restrict__ T,
                                                    const double2 *__restrict__ twf, double2 *__restrict__ S) {
  constexpr int SD = 2 * NSR + 1, ND = SD * SD * SD, FB = 8;
  __shared__ double2 ph[FB][ND];
  const int kk0 = blockIdx.x * FB;
  for (int i = threadIdx.x; i < FB * ND; i += blockDim.x) {
    const int f = i / ND, iD = i % ND;
    const int kk = kk0 + f;
    const int kx = kk % n, ky = (kk / n) % n, kz = kk / (n * n);
    const int Dx = iD % SD - NSR, Dy = (iD / SD) % SD - NSR, Dz = iD / (SD * SD) - NSR;
    int e = (kx * Dx + ky * Dy + kz * Dz) % n;
    e += e < 0 ? n : 0;
    ph[f][iD] = twf[e];
  }
  __syncthreads();
  const int m = threadIdx.x;
  if (m >= nm) return;
  for (int a = 0; a < 8; ++a) {
    double2 acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = make_double2(0.0, 0.0);
    const double *Ta = T + size_t(a) * ND * nm + m;
    for (int iD = 0; iD < ND; ++iD) {
      const double t = Ta[size_t(iD) * nm];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        acc[f].x += t * ph[f][iD].x;
        acc[f].y += t * ph[f][iD].y;
      }
    }
#pragma unroll
    for (int f = 0; f < FB; ++f) S[(size_t(kk0 + f) * 8 + a) * nm + m] = acc[f];
  }
}

// A[E][a] = 4 pi <lambda_E, G_a> - B_E[a], B from the inverse transform.
template <int PO>
__global__ __launch_bounds__(256) void k_adj_finish(int n, int nb, const double *__restrict__ lam,
                                                    const double *__restrict__ gw, const double *__restrict__ Bn,
                                                    double *__restrict__ Aout) {
  constexpr int Q1 = PO + 1;
  const size_t M = size_t(n) * n * n;
  const size_t E = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (E >= size_t(nb) * M) return;
  const int cfg = int(E / M);
  const int el = int(E % M);
  const int ex = el % n, ey = (el / n) % n, ez = el / (n * n);
  const int P = PO * n;
  lam += size_t(cfg) * P * P * P;
  double a1[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int mz = 0; mz < Q1; ++mz) {
    int gz = PO * ez + mz;
    gz -= gz >= P ? P : 0;
    for (int my = 0; my < Q1; ++my) {
      int gy = PO * ey + my;
      gy -= gy >= P ? P : 0;
      const double *row = lam + (size_t(gz) * P + gy) * P;
      for (int mx = 0; mx < Q1; ++mx) {
        int gx = PO * ex + mx;
        gx -= gx >= P ? P : 0;
        const double lv = row[gx];
        const double gx0 = gw[mx], gx1 = gw[Q1 + mx], gy0 = gw[my], gy1 = gw[Q1 + my], gz0 = gw[mz], gz1 = gw[Q1 + mz];
        a1[0] += lv * gx0 * gy0 * gz0;
        a1[1] += lv * gx1 * gy0 * gz0;
        a1[2] += lv * gx0 * gy1 * gz0;
        a1[3] += lv * gx1 * gy1 * gz0;
        a1[4] += lv * gx0 * gy0 * gz1;
        a1[5] += lv * gx1 * gy0 * gz1;
        a1[6] += lv * gx0 * gy1 * gz1;
        a1[7] += lv * gx1 * gy1 * gz1;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) Aout[E * 8 + a] = 4.0 * M_PI * a1[a] - Bn[E * 8 + a];
}

// ------------------------------------------------------------- launchers

bool fft_size_ok(int n) { return n >= 8 && n <= 128 && (n & (n - 1)) == 0; }

size_t spec_freqs(int n) { return size_t(n) * n * (n / 2 + 1); }

namespace {

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

void fft_shape(int n, int nch, int &cc, int &lb) {
  cc = nch;
  while (n * cc > kFftCap || nch % cc != 0) --cc;
  lb = 1;
  while (2 * lb <= n && n * 2 * lb * cc <= kFftCap) lb *= 2;
}

template <bool INV, int EPI, class WT>
void fft_pass(hipStream_t s, int nb, int n, int nch, int axis, const double2 *src, double2 *dst,
              const double2 *tw, const double *phi, WT *W, int po) {
  int cc, lb;
  fft_shape(n, nch, cc, lb);
  const size_t lds = (size_t(n) * lb * cc + n / 2) * sizeof(double2);
  const dim3 grid(unsigned(size_t(nb) * n * (n / lb) * (nch / cc)));
  hipLaunchKernelGGL((k_fft_axis<INV, EPI, WT>), grid, dim3(256), lds, s, n, ilog2(n), nch, cc, lb, axis, src, dst,
                     tw, phi, W, po);
}

// forward 3-D transform: src (real pairs) -> dst, x then y then z
void fft3_forward(hipStream_t s, int nb, int n, int nch, const double2 *src, double2 *dst, const double2 *tw) {
  fft_pass<false, 0, double>(s, nb, n, nch, 0, src, dst, tw, nullptr, nullptr, 0);
  fft_pass<false, 0, double>(s, nb, n, nch, 1, dst, dst, tw, nullptr, nullptr, 0);
  fft_pass<false, 0, double>(s, nb, n, nch, 2, dst, dst, tw, nullptr, nullptr, 0);
}

}  // namespace

void launch_spec_build(hipStream_t s, int n, int nsr, int p, const double *T, const double2 *twf, double2 *S) {
  const int nm = (p + 1) * (p + 1) * (p + 1);
  const dim3 grid(unsigned(spec_freqs(n) / 8));
  switch (nsr) {
    case 1: hipLaunchKernelGGL(k_spec_build<1>, grid, dim3(256), 0, s, n, nm, T, twf, S); break;
    case 2: hipLaunchKernelGGL(k_spec_build<2>, grid, dim3(256), 0, s, n, nm, T, twf, S); break;
    default: hipLaunchKernelGGL(k_spec_build<3>, grid, dim3(256), 0, s, n, nm, T, twf, S); break;
  }
}

template <class WT>
int launch_psi_fft(hipStream_t s, int nb, int n, int p, const double *C, const double2 *S, const double2 *tw,
                   const double *phi, double2 *zc, double2 *z, WT *Wel) {
  if (p != 5 || !fft_size_ok(n)) return -1;
  const int nm = (p + 1) * (p + 1) * (p + 1), nc = nm / 2;
  const int NF = int(spec_freqs(n));
  fft3_forward(s, nb, n, 4, reinterpret_cast<const double2 *>(C), zc, tw);
  const double scale = 1.0 / (double(n) * n * n);
  hipLaunchKernelGGL(k_spec_psi, dim3(unsigned(size_t(nb) * NF)), dim3(128), 0, s, n, NF, nm, S, zc, z, scale);
  fft_pass<true, 0, double>(s, nb, n, nc, 0, z, z, tw, nullptr, nullptr, p);
  fft_pass<true, 0, double>(s, nb, n, nc, 1, z, z, tw, nullptr, nullptr, p);
  fft_pass<true, 1, WT>(s, nb, n, nc, 2, z, z, tw, phi, Wel, p);
  return 0;
}
template int launch_psi_fft<double>(hipStream_t, int, int, int, const double *, const double2 *, const double2 *,
                                    const double *, double2 *, double2 *, double *);
template int launch_psi_fft<float>(hipStream_t, int, int, int, const double *, const double2 *, const double2 *,
                                   const double *, double2 *, double2 *, float *);

int launch_adj_moments_fft(hipStream_t s, int nb, int p, int n, const double *gE, const double2 *S,
                           const double2 *tw, const double *lam, const double *gw, double2 *z, double2 *za,
                           double *A) {
  if (p != 5 || !fft_size_ok(n)) return -1;
  const int nm = (p + 1) * (p + 1) * (p + 1), nc = nm / 2;
  const int NF = int(spec_freqs(n));
  fft3_forward(s, nb, n, nc, reinterpret_cast<const double2 *>(gE), z, tw);
  const double scale = 1.0 / (double(n) * n * n);
  hipLaunchKernelGGL(k_spec_adj, dim3(unsigned(size_t(nb) * NF)), dim3(128), 0, s, n, NF, nm, S, z, za, scale);
  fft_pass<true, 0, double>(s, nb, n, 4, 0, za, za, tw, nullptr, nullptr, 0);
  fft_pass<true, 0, double>(s, nb, n, 4, 1, za, za, tw, nullptr, nullptr, 0);
  fft_pass<true, 0, double>(s, nb, n, 4, 2, za, za, tw, nullptr, nullptr, 0);
  const size_t ne = size_t(nb) * n * n * n;
  hipLaunchKernelGGL(k_adj_finish<5>, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, n, nb, lam, gw,
                     reinterpret_cast<const double *>(za), A);
  return 0;
}

}  // namespace fep3m
