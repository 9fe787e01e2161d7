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
// element for the direct sums; the work becomes memory-bound.
//
// Layout: every transformed field is [config][z][y][x][channel] complex
// (double2), channel fastest, where two consecutive real channels form one
// complex channel: the moments C[E][8] are 4 complex channels in place, the
// node fields [E][216] are 108.  One complex FFT of the pair (X_2c + i X_2c+1)
// transforms both real channels; X^_2c(k) = (Z(k) + conj Z(-k)) / 2 and
// X^_2c+1(k) = (Z(k) - conj Z(-k)) / 2i separate them in the products, which
// also pack their two real outputs the same way, so the inverse transforms
// return real pairs directly.  The tables are symmetric under the three axis
// reflections, so the spectrum is kept for one octant of frequencies
// (0 <= k_x, k_y, k_z <= n/2: 0.99 GB at n = 64) and each product block
// handles the orbit of one octant frequency (which holds -k as well).  With
// forces both products run in the same blocks: one read of the spectrum.
//
// FFTs: one kernel per axis, decimation in time in LDS (radix-2 stages
// taken two at a time).  A block holds lb lines x cc channels of length n
// (at most 2048 complex values):
// rows of cc consecutive channels (and lb consecutive elements across the
// line for the y and z passes) are contiguous in memory.  Twiddles come from
// a table computed on the host.  n is a power of two, 8 .. 64.
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

}  // namespace

// Block shape of an FFT pass: cc channels (a divisor of nch) x lb lines of
// length n, at most kFftCap complex values.
constexpr int fft_cc(int n, int nch) {
  int cc = nch;
  while (n * cc > kFftCap || nch % cc != 0) --cc;
  return cc;
}
constexpr int fft_lb(int n, int nch) {
  const int cc = fft_cc(n, nch);
  int lb = 1;
  while (2 * lb <= n && n * 2 * lb * cc <= kFftCap) lb *= 2;
  return lb;
}

// One axis of a batched 3-D FFT over [cfg][z][y][x][NCH] complex values,
// n = 2^LOGN.  EPI 0: store the transformed values to dst (src == dst
// allowed: a block reads all its values before it writes).  EPI 1 (last
// inverse pass of the field): the values are (Psi_2c, Psi_2c+1) of element
// E; store W_E[m] = phi(node of m) - Psi_m to Wout (float64 or float32),
// phi the order-po mesh potential.
template <int LOGN, int NCH, bool INV, int EPI, class WT>
__global__ __launch_bounds__(256) void k_fft_axis(int axis, const double2 *src, double2 *dst,
                                                  const double2 *__restrict__ tw, const double *__restrict__ phi,
                                                  WT *__restrict__ Wout, int po) {
  constexpr int N = 1 << LOGN, CC = fft_cc(N, NCH), LB = fft_lb(N, NCH);
  constexpr int U = LB * CC, TOT = N * U;
  constexpr int NCHUNK = NCH / CC, NG = N / LB;
  __shared__ double2 buf[TOT];   // [j][u], u = l CC + c
  __shared__ double2 tws[N / 2];
  int b = blockIdx.x;
  const int chunk = b % NCHUNK;
  b /= NCHUNK;
  const int g = b % NG;
  b /= NG;
  const int outer = b % N;
  const int cfg = b / N;
  size_t sj, sl, so;
  if (axis == 0) { sj = NCH; sl = size_t(N) * NCH; so = size_t(N) * N * NCH; }
  else if (axis == 1) { sj = size_t(N) * NCH; sl = NCH; so = size_t(N) * N * NCH; }
  else { sj = size_t(N) * N * NCH; sl = NCH; so = size_t(N) * NCH; }
  const size_t base = size_t(cfg) * N * N * N * NCH + size_t(outer) * so + size_t(g) * LB * sl + size_t(chunk) * CC;
  const int tid = threadIdx.x;
  // position (j, l, c) of value i: the thread order follows memory
  auto coords = [&](int i, int &j, int &l, int &c) {
    c = i % CC;
    const int r = i / CC;
    if (axis == 0) { j = r % N; l = r / N; } else { l = r % LB; j = r / LB; }
  };
  if (tid < N / 2) tws[tid] = tw[tid];
  for (int i = tid; i < TOT; i += 256) {   // stored in bit-reversed order of j
    int j, l, c;
    coords(i, j, l, c);
    buf[int(__brev(unsigned(j)) >> (32 - LOGN)) * U + l * CC + c] = src[base + j * sj + l * sl + c];
  }
  __syncthreads();
  // Radix-2 stages (half-size h = 2^s, twiddle W_2h^pos), taken two at a
  // time: one pass over LDS does stages s and s + 1 on the four values
  // j0 + {0, h, 2h, 3h} (the same operations in the same order, so the
  // result equals the stage-by-stage one); an odd count starts with a single
  // stage.
  if (LOGN & 1) {
    for (int t = tid; t < (N / 2) * U; t += 256) {   // s = 0: twiddle 1
      const int u = t % U, j0 = 2 * (t / U);
      const double2 x0 = buf[j0 * U + u], x1 = cmul(buf[(j0 + 1) * U + u], tws[0]);
      buf[j0 * U + u] = cadd(x0, x1);
      buf[(j0 + 1) * U + u] = csub(x0, x1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = LOGN & 1; s < LOGN; s += 2) {
    const int h = 1 << s;
    for (int t = tid; t < (N / 4) * U; t += 256) {
      const int u = t % U, bf = t / U;
      const int pos = bf & (h - 1);
      const int j0 = ((bf >> s) << (s + 2)) + pos;
      double2 w1 = tws[pos << (LOGN - 1 - s)], w2 = tws[pos << (LOGN - 2 - s)],
              w3 = tws[(pos + h) << (LOGN - 2 - s)];
      if (INV) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
      const double2 x0 = buf[j0 * U + u], x1 = buf[(j0 + h) * U + u];
      const double2 x2 = buf[(j0 + 2 * h) * U + u], x3 = buf[(j0 + 3 * h) * U + u];
      const double2 t1 = cmul(x1, w1), t3 = cmul(x3, w1);
      const double2 a0 = cadd(x0, t1), a1 = csub(x0, t1), a2 = cadd(x2, t3), a3 = csub(x2, t3);
      const double2 t2 = cmul(a2, w2), t4 = cmul(a3, w3);
      buf[j0 * U + u] = cadd(a0, t2);
      buf[(j0 + h) * U + u] = cadd(a1, t4);
      buf[(j0 + 2 * h) * U + u] = csub(a0, t2);
      buf[(j0 + 3 * h) * U + u] = csub(a1, t4);
    }
    __syncthreads();
  }
  if (EPI == 0) {
    for (int i = tid; i < TOT; i += 256) {
      int j, l, c;
      coords(i, j, l, c);
      dst[base + j * sj + l * sl + c] = buf[j * U + l * CC + c];
    }
  } else {
    const int Q1 = po + 1, NM = Q1 * Q1 * Q1, P = po * N;
    const size_t M = size_t(N) * N * N;
    phi += size_t(cfg) * P * P * P;
    for (int i = tid; i < TOT; i += 256) {
      int j, l, c;
      coords(i, j, l, c);
      int ex, ey, ez;
      const int lc = g * LB + l;
      if (axis == 0) { ex = j; ey = lc; ez = outer; }
      else if (axis == 1) { ey = j; ex = lc; ez = outer; }
      else { ez = j; ex = lc; ey = outer; }
      const double2 v = buf[j * U + l * CC + c];
      const size_t E = size_t(cfg) * M + (size_t(ez) * N + ey) * N + ex;
      const int ch = chunk * CC + c;
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

// Spectrum products over the orbit of one octant frequency k (0 <= k_x,
// k_y, k_z <= n/2) under the reflections of the axes whose component is
// neither 0 nor n/2 (pm): the up to 8 frequencies R k, among them -k.  The
// tables are symmetric under each axis reflection R (node m -> R m, offset
// D -> R D, moment a -> (-1)^(a.R) a), so S[a][m](R k) = (-1)^(a.R)
// S[a][R m](k): one stored row of 8 x 216 values serves the whole orbit.
//   PSI: Zpsi(R k)[c] = (Psi^_2c + i Psi^_2c+1)(R k) * scale
//   ADJ: ZA(R k)[j] = (B^_2j + i B^_2j+1)(R k) * scale
// Moments are indexed a = a_x + 2 a_y + 4 a_z (each 0 or 1), nodes
// m = m_x + 6 (m_y + 6 m_z).
constexpr int kOrbitThreads = 512;

template <bool PSI, bool ADJ>
__global__ __launch_bounds__(kOrbitThreads) void k_spec_orbit(int n, int NO, const double2 *__restrict__ S,
                                                    const double2 *__restrict__ ZC, double2 *__restrict__ Zpsi,
                                                    const double2 *__restrict__ Zg, double2 *__restrict__ ZA,
                                                    double scale) {
  constexpr int Q1 = 6, NM = Q1 * Q1 * Q1, NC = NM / 2, NT = kOrbitThreads, NQ = NT / 64;
  static_assert(NM % NQ == 0 && NQ * 64 <= 8 * NM, "node split of the transposed product");
  __shared__ double2 Ss[8 * NM + 1];   // one spare slot
  __shared__ double2 Cs[8][8];
  __shared__ double2 Gs[ADJ ? 8 * NM : 1];   // reused for the partial sums
  const int H = n / 2 + 1;
  const int ko = blockIdx.x % NO, cfg = blockIdx.x / NO;
  const int kx = ko % H, ky = (ko / H) % H, kz = ko / (H * H);
  int pm = 0;
  if (kx != 0 && 2 * kx != n) pm |= 1;
  if (ky != 0 && 2 * ky != n) pm |= 2;
  if (kz != 0 && 2 * kz != n) pm |= 4;
  auto fidx = [&](int r) {
    const int x = (r & 1) ? n - kx : kx, y = (r & 2) ? n - ky : ky, z = (r & 4) ? n - kz : kz;
    return size_t((z * n + y) * n + x);
  };
  auto refl = [](int m, int r) {
    int mx = m % Q1, my = (m / Q1) % Q1, mz = m / (Q1 * Q1);
    if (r & 1) mx = Q1 - 1 - mx;
    if (r & 2) my = Q1 - 1 - my;
    if (r & 4) mz = Q1 - 1 - mz;
    return (mz * Q1 + my) * Q1 + mx;
  };
  const size_t M = size_t(n) * n * n;
  const int tid = threadIdx.x;
  const double2 *Sk = S + size_t(ko) * 8 * NM;
  {   // all loads of the row in flight before the LDS stores
    constexpr int KS = (8 * NM + NT - 1) / NT;
    double2 v[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) v[k] = Sk[min(tid + NT * k, 8 * NM - 1)];   // clamped: no branch per load
    asm volatile("" ::: "memory");   // compiler fence: all loads issue before the stores
#pragma unroll
    for (int k = 0; k < KS; ++k) Ss[min(tid + NT * k, 8 * NM)] = v[k];   // lanes past the end: spare slot
  }
  if constexpr (PSI) if (tid < 64) {   // C^_a at each orbit frequency, from Z(f) and Z(-f)
    const int r = tid >> 3, a = tid & 7;
    if ((r & ~pm) == 0) {
      const double2 z = ZC[(size_t(cfg) * M + fidx(r)) * 4 + (a >> 1)];
      const double2 zm = ZC[(size_t(cfg) * M + fidx(r ^ pm)) * 4 + (a >> 1)];
      Cs[r][a] = (a & 1) ? make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x))
                         : make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
    }
  }
  if constexpr (ADJ) {
    constexpr int KG = (8 * NC + NT - 1) / NT;
    double2 z[KG], zm[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) {   // unconditional loads (frequencies outside the orbit read k itself)
      const int i = min(tid + NT * k, 8 * NC - 1), r = (i / NC) & pm, c = i % NC;
      z[k] = Zg[(size_t(cfg) * M + fidx(r)) * NC + c];
      zm[k] = Zg[(size_t(cfg) * M + fidx(r ^ pm)) * NC + c];
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < KG; ++k) {   // slots outside the orbit are written but never read
      const int i = min(tid + NT * k, 8 * NC - 1), r = i / NC, c = i % NC;
      Gs[r * NM + 2 * c] = make_double2(0.5 * (z[k].x + zm[k].x), 0.5 * (z[k].y - zm[k].y));
      Gs[r * NM + 2 * c + 1] = make_double2(0.5 * (z[k].y + zm[k].y), -0.5 * (z[k].x - zm[k].x));
    }
  }
  __syncthreads();
  if constexpr (PSI) {
    for (int i = tid; i < 8 * NC; i += NT) {
      const int r = i / NC, c = i % NC;
      if (r & ~pm) continue;
      const int m0 = refl(2 * c, r), m1 = refl(2 * c + 1, r);
      double2 P0 = make_double2(0.0, 0.0), P1 = make_double2(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const double sg = (__popc(a & r) & 1) ? -1.0 : 1.0;
        const double2 ch = make_double2(sg * Cs[r][a].x, sg * Cs[r][a].y);
        P0 = cadd(P0, cmul(Ss[a * NM + m0], ch));
        P1 = cadd(P1, cmul(Ss[a * NM + m1], ch));
      }
      Zpsi[(size_t(cfg) * M + fidx(r)) * NC + c] = make_double2((P0.x - P1.y) * scale, (P0.y + P1.x) * scale);
    }
  }
  if constexpr (ADJ) {
    // 64 outputs (orbit member r, moment a) x NQ node ranges; the partial
    // sums then go to Gs (no longer read) and are added in a fixed order
    const int o = tid & 63, q = tid >> 6;
    const int r = o >> 3, a = o & 7;
    double2 acc = make_double2(0.0, 0.0);
    if ((r & ~pm) == 0) {
      constexpr int MQ = NM / NQ;
      for (int m = q * MQ; m < (q + 1) * MQ; ++m) acc = cadd(acc, cmulc(Ss[a * NM + refl(m, r)], Gs[r * NM + m]));
      if (__popc(a & r) & 1) acc = make_double2(-acc.x, -acc.y);
    }
    __syncthreads();
    double2 *red = Gs;   // [q][64]
    red[q * 64 + o] = acc;
    __syncthreads();
    if (tid < 32) {
      const int rr = tid >> 2, j = tid & 3;
      if ((rr & ~pm) == 0) {
        double2 A0 = red[rr * 8 + 2 * j], A1 = red[rr * 8 + 2 * j + 1];
#pragma unroll
        for (int k = 1; k < NQ; ++k) {
          A0 = cadd(A0, red[k * 64 + rr * 8 + 2 * j]);
          A1 = cadd(A1, red[k * 64 + rr * 8 + 2 * j + 1]);
        }
        ZA[(size_t(cfg) * M + fidx(rr)) * 4 + j] = make_double2((A0.x - A1.y) * scale, (A0.y + A1.x) * scale);
      }
    }
  }
}

// Table spectrum S[ko][a][m] at the octant frequencies ko = k_x + H (k_y +
// H k_z), H = n/2 + 1: 8 frequencies per block, one thread per node m, the
// phases exp(-2 pi i k.D / n) = tw[(k.D) mod n] of the block's frequencies
// in LDS.
template <int NSR>
__global__ __launch_bounds__(256) void k_spec_build(int n, int NO, int nm, const double *__restrict__ T,
                                                    const double2 *__restrict__ twf, double2 *__restrict__ S) {
  constexpr int SD = 2 * NSR + 1, ND = SD * SD * SD, FB = 8;
  __shared__ double2 ph[FB][ND];
  const int H = n / 2 + 1;
  const int ko0 = blockIdx.x * FB;
  for (int i = threadIdx.x; i < FB * ND; i += blockDim.x) {
    const int f = i / ND, iD = i % ND;
    const int ko = min(ko0 + f, NO - 1);
    const int kx = ko % H, ky = (ko / H) % H, kz = ko / (H * H);
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
    for (int f = 0; f < FB; ++f)
      if (ko0 + f < NO) S[(size_t(ko0 + f) * 8 + a) * nm + m] = acc[f];
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

bool fft_size_ok(int n) { return n >= 8 && n <= 64 && (n & (n - 1)) == 0; }

size_t spec_freqs(int n) { return size_t(n / 2 + 1) * (n / 2 + 1) * (n / 2 + 1); }

namespace {

template <int LOGN, int NCH, bool INV, int EPI, class WT>
void fft_launch(hipStream_t s, int nb, int axis, const double2 *src, double2 *dst, const double2 *tw,
                const double *phi, WT *W, int po) {
  constexpr int N = 1 << LOGN, CC = fft_cc(N, NCH), LB = fft_lb(N, NCH);
  const dim3 grid(unsigned(size_t(nb) * N * (N / LB) * (NCH / CC)));
  hipLaunchKernelGGL((k_fft_axis<LOGN, NCH, INV, EPI, WT>), grid, dim3(256), 0, s, axis, src, dst, tw, phi, W, po);
}

template <int NCH, bool INV, int EPI, class WT>
void fft_pass_n(hipStream_t s, int nb, int n, int axis, const double2 *src, double2 *dst, const double2 *tw,
                const double *phi, WT *W, int po) {
  switch (n) {
    case 8: fft_launch<3, NCH, INV, EPI, WT>(s, nb, axis, src, dst, tw, phi, W, po); break;
    case 16: fft_launch<4, NCH, INV, EPI, WT>(s, nb, axis, src, dst, tw, phi, W, po); break;
    case 32: fft_launch<5, NCH, INV, EPI, WT>(s, nb, axis, src, dst, tw, phi, W, po); break;
    default: fft_launch<6, NCH, INV, EPI, WT>(s, nb, axis, src, dst, tw, phi, W, po); break;
  }
}

// nch: 4 (moments) or 108 (node fields); EPI 1 only for node fields
template <bool INV, int EPI, class WT>
void fft_pass(hipStream_t s, int nb, int n, int nch, int axis, const double2 *src, double2 *dst,
              const double2 *tw, const double *phi, WT *W, int po) {
  if (EPI == 0 && nch == 4)
    fft_pass_n<4, INV, 0, WT>(s, nb, n, axis, src, dst, tw, phi, W, po);
  else
    fft_pass_n<108, INV, EPI, WT>(s, nb, n, axis, src, dst, tw, phi, W, po);
}

template <bool INV>
int fft_pass_nodes(hipStream_t s, int nb, int n, int nch, int axis, double2 *z, const double2 *tw) {
  switch (nch) {
    case 27: fft_pass_n<27, INV, 0, double>(s, nb, n, axis, z, z, tw, nullptr, nullptr, 0); return 0;
    case 64: fft_pass_n<64, INV, 0, double>(s, nb, n, axis, z, z, tw, nullptr, nullptr, 0); return 0;
    case 125: fft_pass_n<125, INV, 0, double>(s, nb, n, axis, z, z, tw, nullptr, nullptr, 0); return 0;
    case 216: fft_pass_n<216, INV, 0, double>(s, nb, n, axis, z, z, tw, nullptr, nullptr, 0); return 0;
    default: return -1;
  }
}

// forward 3-D transform: src (real pairs) -> dst, x then y then z
void fft3_forward(hipStream_t s, int nb, int n, int nch, const double2 *src, double2 *dst, const double2 *tw) {
  fft_pass<false, 0, double>(s, nb, n, nch, 0, src, dst, tw, nullptr, nullptr, 0);
  fft_pass<false, 0, double>(s, nb, n, nch, 1, dst, dst, tw, nullptr, nullptr, 0);
  fft_pass<false, 0, double>(s, nb, n, nch, 2, dst, dst, tw, nullptr, nullptr, 0);
}

}  // namespace

int launch_fft3_nodes(hipStream_t s, int nb, int n, int nch, double2 *z, const double2 *tw, bool inverse) {
  if (!fft_size_ok(n)) return -1;
  for (int a = 0; a < 3; ++a) {
    const int axis = inverse ? 2 - a : a;
    if ((inverse ? fft_pass_nodes<true>(s, nb, n, nch, axis, z, tw) : fft_pass_nodes<false>(s, nb, n, nch, axis, z, tw)) != 0)
      return -1;
  }
  return 0;
}

void launch_spec_build(hipStream_t s, int n, int nsr, int p, const double *T, const double2 *twf, double2 *S) {
  const int nm = (p + 1) * (p + 1) * (p + 1);
  const int NO = int(spec_freqs(n));
  const dim3 grid(unsigned((NO + 7) / 8));
  switch (nsr) {
    case 1: hipLaunchKernelGGL(k_spec_build<1>, grid, dim3(256), 0, s, n, NO, nm, T, twf, S); break;
    case 2: hipLaunchKernelGGL(k_spec_build<2>, grid, dim3(256), 0, s, n, NO, nm, T, twf, S); break;
    default: hipLaunchKernelGGL(k_spec_build<3>, grid, dim3(256), 0, s, n, NO, nm, T, twf, S); break;
  }
}

int launch_near_fft(hipStream_t s, int nb, int n, int p, const double *C, const double *gE, const double2 *S,
                    const double2 *tw, double2 *zc, double2 *zpsi, double2 *zg, double2 *za) {
  if (p != 5 || !fft_size_ok(n) || (!C && !gE)) return -1;
  const int nc = (p + 1) * (p + 1) * (p + 1) / 2;
  const int NO = int(spec_freqs(n));
  const double scale = 1.0 / (double(n) * n * n);
  if (C) fft3_forward(s, nb, n, 4, reinterpret_cast<const double2 *>(C), zc, tw);
  if (gE) fft3_forward(s, nb, n, nc, reinterpret_cast<const double2 *>(gE), zg, tw);
  const dim3 grid(unsigned(size_t(nb) * NO));
  if (C && gE)
    hipLaunchKernelGGL((k_spec_orbit<true, true>), grid, dim3(kOrbitThreads), 0, s, n, NO, S, zc, zpsi, zg, za, scale);
  else if (C)
    hipLaunchKernelGGL((k_spec_orbit<true, false>), grid, dim3(kOrbitThreads), 0, s, n, NO, S, zc, zpsi, zg, za, scale);
  else
    hipLaunchKernelGGL((k_spec_orbit<false, true>), grid, dim3(kOrbitThreads), 0, s, n, NO, S, zc, zpsi, zg, za, scale);
  if (gE)
    for (int axis = 0; axis < 3; ++axis) fft_pass<true, 0, double>(s, nb, n, 4, axis, za, za, tw, nullptr, nullptr, 0);
  return 0;
}

template <class WT>
int launch_psi_fft_finish(hipStream_t s, int nb, int n, int p, const double2 *tw, const double *phi, double2 *zpsi,
                          WT *Wel) {
  if (p != 5 || !fft_size_ok(n)) return -1;
  const int nc = (p + 1) * (p + 1) * (p + 1) / 2;
  // z, y, then x with the W epilogue: along x the mesh potential is read in
  // contiguous rows (nodes p e_x + m_x) and W in runs of one element's nodes
  fft_pass<true, 0, double>(s, nb, n, nc, 2, zpsi, zpsi, tw, nullptr, nullptr, p);
  fft_pass<true, 0, double>(s, nb, n, nc, 1, zpsi, zpsi, tw, nullptr, nullptr, p);
  fft_pass<true, 1, WT>(s, nb, n, nc, 0, zpsi, zpsi, tw, phi, Wel, p);
  return 0;
}
template int launch_psi_fft_finish<double>(hipStream_t, int, int, int, const double2 *, const double *, double2 *,
                                           double *);
template int launch_psi_fft_finish<float>(hipStream_t, int, int, int, const double2 *, const double *, double2 *,
                                          float *);

int launch_adj_fft_finish(hipStream_t s, int nb, int n, int p, const double *lam, const double *gw, const double2 *za,
                          double *A) {
  if (p != 5 || !fft_size_ok(n)) return -1;
  const size_t ne = size_t(nb) * n * n * n;
  hipLaunchKernelGGL(k_adj_finish<5>, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, n, nb, lam, gw,
                     reinterpret_cast<const double *>(za), A);
  return 0;
}

}  // namespace fep3m
