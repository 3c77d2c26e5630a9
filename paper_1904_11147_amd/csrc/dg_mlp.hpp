// Learned troubled-cell indicator: features, MLP forward/backward with BF16
// MFMA (FP32 accumulate), Adam, and the indicator kernel of the limiter.
// Included into dg_kernels.hip (inside its anonymous namespace), so it shares
// the coefficient tables, the boundary handling and the TVB decision.
//
// Network: x (F features, padded to KP, bf16) -> h1 = relu(W1 x + b1) (64)
// -> h2 = relu(W2 h1 + b2) (64) -> z = w3 . h2 + b3 -> p = sigmoid(z).
// Weights bf16, biases and accumulation fp32.
//
// MFMA v_mfma_f32_16x16x16_bf16 register layout (wave64, lane l, r = l % 16,
// g = l / 16):  A (16 x 16, rows x k):   lane holds A[r][4g .. 4g+3]
//               B (16 x 16, k x cols):   lane holds B[4g .. 4g+3][r]
//               D (16 x 16, rows x cols): lane holds D[4g + i][r], i = 0..3.

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kHidden = 64;

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// the same rounding (to nearest even) by the hardware conversion, for the limiter's inference
__device__ inline uint16_t f2bf_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ inline f32x4_t mfma16(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ inline bf16x4_t pack4(float a, float b, float c, float d) {
  bf16x4_t v;
  v[0] = (short)f2bf(a);
  v[1] = (short)f2bf(b);
  v[2] = (short)f2bf(c);
  v[3] = (short)f2bf(d);
  return v;
}

__device__ inline bf16x4_t load4(const uint16_t *p) { return *reinterpret_cast<const bf16x4_t *>(p); }

// Offsets into the bf16 weight buffer: W1 [64][KP] | W2 [64][64] | W2T [64][64] | w3 [64] | W1P.
//
// W1P is W1 rearranged for the limiter's inference kernel, where each of the
// four lane groups of an MFMA fragment handles one of the four conserved
// variables: the F = 4 FV features split into four per-variable blocks of FV,
// each padded to BV = 4 ceil(FV / 4) (so 4 BV = KP for FV = 5 (N+1)^2), and
// stored as [nb][kb][lane][K] A-fragments: element e of lane (r, g) of
// k-block kb and output block nb is W1[16 nb + r][g FV + K kb + e] (zero in
// the padding), with K = 8 (the 16x16x32 MFMA) when BV is a multiple of 8,
// else K = 4 (16x16x16).  Defined when F is a multiple of 4 with 4 BV = KP.
struct MlpLayout {
  int F, KP;
  __host__ __device__ long w1() const { return 0; }
  __host__ __device__ long w2() const { return (long)kHidden * KP; }
  __host__ __device__ long w2t() const { return w2() + kHidden * kHidden; }
  __host__ __device__ long w3() const { return w2t() + kHidden * kHidden; }
  __host__ __device__ long w1p() const { return w3() + kHidden; }
  __host__ __device__ long nbf16() const { return w1p() + (long)kHidden * KP; }
  __host__ __device__ int fv() const { return F / 4; }
  __host__ __device__ int bv() const { return (F / 4 + 3) / 4 * 4; }
  __host__ __device__ bool has_w1p() const { return F % 4 == 0 && 4 * bv() == KP; }
  __host__ __device__ long npad() const { return has_w1p() ? (long)kHidden * 4 * (bv() - fv()) : 0; }
  __host__ __device__ int frag() const { return bv() % 8 == 0 ? 8 : 4; }
  // W1P position of W1[o][v FV + f]
  __host__ __device__ long w1p_at(int o, int v, int f) const {
    const int K = frag(), KB = bv() / K;
    return w1p() + ((long)((o / 16) * KB + f / K) * 64 + v * 16 + o % 16) * K + f % K;
  }
  // master fp32: W1 [64][F] | W2 [64][64] | w3 [64] | b1 [64] | b2 [64] | b3
  __host__ __device__ long mW2() const { return (long)kHidden * F; }
  __host__ __device__ long mw3() const { return mW2() + kHidden * kHidden; }
  __host__ __device__ long mb1() const { return mw3() + kHidden; }
  __host__ __device__ long mb2() const { return mb1() + kHidden; }
  __host__ __device__ long mb3() const { return mb2() + kHidden; }
  __host__ __device__ long nmaster() const { return mb3() + 1; }
};

// One 16-sample tile through the network.  loadA(kb) returns the lane's A
// fragment of the input rows (row r, features 16 kb + 4g ..).  lds is a
// 16 x 64 bf16 scratch.  Outputs in D layout: h1, h2 (post-ReLU, fp32) and
// z for samples 4g + i (the same in all 16 lanes of group g).
template <int KP, typename LoadA>
__device__ inline void mlp_tile_forward(LoadA loadA, const uint16_t *__restrict__ W, const float *__restrict__ M,
                                        const MlpLayout &lay, uint16_t *lds, f32x4_t (&h1)[4], f32x4_t (&h2)[4],
                                        float (&z)[4]) {
  const int lane = __lane_id(), r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) h1[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < KP / 16; ++kb) {
    const bf16x4_t a = loadA(kb);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      h1[nt] = mfma16(a, load4(W + lay.w1() + (long)(16 * nt + r) * KP + 16 * kb + 4 * g), h1[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const float b = M[lay.mb1() + 16 * nt + r];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h1[nt][i] = fmaxf(h1[nt][i] + b, 0.f);
      lds[(4 * g + i) * kHidden + 16 * nt + r] = f2bf(h1[nt][i]);
    }
  }
  __syncthreads();  // one wavefront per block: orders the LDS tile
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) h2[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const bf16x4_t a = load4(lds + r * kHidden + 16 * kb + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      h2[nt] = mfma16(a, load4(W + lay.w2() + (16 * nt + r) * kHidden + 16 * kb + 4 * g), h2[nt]);
  }
  __syncthreads();  // the scratch tile may be rewritten by the caller next
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const float b = M[lay.mb2() + 16 * nt + r];
    const float w3 = bf2f(W[lay.w3() + 16 * nt + r]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h2[nt][i] = fmaxf(h2[nt][i] + b, 0.f);
      part[i] += bf2f(f2bf(h2[nt][i])) * w3;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float s = part[i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    z[i] = s + M[lay.mb3()];
  }
}

// Features of cell (i, j) for variable v written as bf16 into dst[0..5*NM)
// (and fp32 into dst32 when given): cells C, W, E, S, N in that order, each
// with its modes; mode-0 entries shifted by the centre's mode 0; all scaled
// by max(max |entry|, M hx^2).
template <int N, int NV>
__device__ inline void cell_features(const double *__restrict__ u, const Geometry &g, int i, int j, int v,
                                     uint16_t *dst, float *dst32) {
  constexpr int NP = N + 1, NM = NP * NP;
  const long plane = (long)g.nx * g.ny;
  double f[5 * NM];
  const int di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const CellIdx ci = map_cell(g, i + di[c], j + dj[c]);
#pragma unroll
    for (int q = 0; q < NM; ++q) f[c * NM + q] = cell_mode<NP, NM, 2>(u, plane, g, ci, v, q);
  }
  const double c0 = f[0];
  double mx = g.tvb_Mx;
#pragma unroll
  for (int c = 0; c < 5; ++c) f[c * NM] -= c0;
#pragma unroll
  for (int k = 0; k < 5 * NM; ++k) mx = fmax(mx, fabs(f[k]));
  const double inv = 1.0 / mx;
#pragma unroll
  for (int k = 0; k < 5 * NM; ++k) {
    const float x = (float)(f[k] * inv);
    if (dst) dst[k] = f2bf(x);
    if (dst32) dst32[k] = x;
  }
}

template <int N, int NV>
__global__ __launch_bounds__(kBlock) void k_mlp_features(const double *__restrict__ u, Geometry g, float *f32,
                                                         uint16_t *bf, int KP) {
  constexpr int NM = (N + 1) * (N + 1), F = 5 * NM * NV;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (long)g.nx * g.ny) return;
  const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
#pragma unroll 1
  for (int v = 0; v < NV; ++v)
    cell_features<N, NV>(u, g, i, j, v, bf ? bf + cell * KP + v * 5 * NM : nullptr,
                         f32 ? f32 + cell * F + v * 5 * NM : nullptr);
  if (bf)
    for (int k = F; k < KP; ++k) bf[cell * KP + k] = 0;
}

// Inference: p for n samples (rows of x, KP bf16 each).  One wavefront per
// 16-sample tile.
template <int KP>
__global__ __launch_bounds__(64) void k_mlp_forward(const uint16_t *__restrict__ x, int n, const uint16_t *W,
                                                    const float *M, MlpLayout lay, float *p) {
  __shared__ uint16_t lds[16 * kHidden];
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const long s0 = (long)blockIdx.x * 16;
  auto loadA = [&](int kb) -> bf16x4_t {
    const long row = s0 + r;
    if (row >= n) return bf16x4_t{0, 0, 0, 0};
    return load4(x + row * KP + 16 * kb + 4 * g);
  };
  f32x4_t h1[4], h2[4];
  float z[4];
  mlp_tile_forward<KP>(loadA, W, M, lay, lds, h1, h2, z);
  if (r == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long s = s0 + 4 * g + i;
      if (s < n) p[s] = 1.f / (1.f + __expf(-z[i]));
    }
}

// Training, part 1: forward and backward of each 16-sample tile; dW2, b2,
// w3, b3, b1 gradients accumulated per wavefront and added atomically; dh1
// (bf16, [n][64]) stored for the dW1 kernel; loss summed atomically.
template <int KP>
__global__ __launch_bounds__(64) void k_mlp_train_tiles(const uint16_t *__restrict__ x, const float *__restrict__ y,
                                                        const float *__restrict__ wgt, int n, const uint16_t *W,
                                                        const float *M, MlpLayout lay, float *G, uint16_t *dh1_out,
                                                        float *loss) {
  __shared__ uint16_t lds[16 * kHidden];
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int ntiles = (n + 15) / 16;
  const float inv_n = 1.0f / (float)n;
  f32x4_t gW2[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};
  float gb3 = 0.f, lsum = 0.f;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long s0 = (long)t * 16;
    auto loadA = [&](int kb) -> bf16x4_t {
      const long row = s0 + r;
      if (row >= n) return bf16x4_t{0, 0, 0, 0};
      return load4(x + row * KP + 16 * kb + 4 * g);
    };
    f32x4_t h1[4], h2[4];
    float z[4];
    mlp_tile_forward<KP>(loadA, W, M, lay, lds, h1, h2, z);
    float dz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long s = s0 + 4 * g + i;
      if (s < n) {
        const float yy = y[s], ww = wgt[s];
        const float pp = 1.f / (1.f + __expf(-z[i]));
        dz[i] = ww * (pp - yy) * inv_n;
        // log(1 + e^z) - y z, stable
        const float sp = fmaxf(z[i], 0.f) + log1pf(__expf(-fabsf(z[i])));
        if (r == 0) lsum += ww * (sp - yy * z[i]) * inv_n;
      } else {
        dz[i] = 0.f;
      }
    }
    // layer 3 and dh2 (D layout), w3 gradient
    f32x4_t dh2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const float w3 = bf2f(W[lay.w3() + 16 * nt + r]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gw3[nt] += dz[i] * bf2f(f2bf(h2[nt][i]));
        dh2[nt][i] = h2[nt][i] > 0.f ? dz[i] * w3 : 0.f;
        gb2[nt] += dh2[nt][i];
      }
    }
    if (r == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) gb3 += dz[i];
    // dW2 += dh2^T h1: both operands are already in the D layout
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x4_t a = pack4(dh2[mt][0], dh2[mt][1], dh2[mt][2], dh2[mt][3]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        gW2[mt][nt] = mfma16(a, pack4(h1[nt][0], h1[nt][1], h1[nt][2], h1[nt][3]), gW2[mt][nt]);
    }
    // dh1 = (dh2 W2) . [h1 > 0]: dh2 to the A layout through LDS, W2^T rows for B
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) lds[(4 * g + i) * kHidden + 16 * nt + r] = f2bf(dh2[nt][i]);
    __syncthreads();
    f32x4_t dh1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) dh1[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x4_t a = load4(lds + r * kHidden + 16 * kb + 4 * g);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        dh1[nt] = mfma16(a, load4(W + lay.w2t() + (16 * nt + r) * kHidden + 16 * kb + 4 * g), dh1[nt]);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float d = h1[nt][i] > 0.f ? dh1[nt][i] : 0.f;
        gb1[nt] += d;
        const long s = s0 + 4 * g + i;
        if (s < n) dh1_out[s * kHidden + 16 * nt + r] = f2bf(d);
      }
  }
  // reduce over the four lane groups and add
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    float a1 = gb1[nt], a2 = gb2[nt], a3 = gw3[nt];
    a1 += __shfl_xor(a1, 16);
    a1 += __shfl_xor(a1, 32);
    a2 += __shfl_xor(a2, 16);
    a2 += __shfl_xor(a2, 32);
    a3 += __shfl_xor(a3, 16);
    a3 += __shfl_xor(a3, 32);
    if (g == 0) {
      atomicAdd(&G[lay.mb1() + 16 * nt + r], a1);
      atomicAdd(&G[lay.mb2() + 16 * nt + r], a2);
      atomicAdd(&G[lay.mw3() + 16 * nt + r], a3);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) atomicAdd(&G[lay.mW2() + (16 * mt + 4 * g + i) * kHidden + 16 * nt + r], gW2[mt][nt][i]);
  float b3 = gb3, ls = lsum;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    b3 += __shfl_xor(b3, o);
    ls += __shfl_xor(ls, o);
  }
  if (lane == 0) {
    atomicAdd(&G[lay.mb3()], b3);
    atomicAdd(loss, ls);
  }
}

// Training, part 2: dW1 += dh1^T x over a chunk of samples (split-K), one
// wavefront per (chunk, 64-column group of the padded input).
template <int KP>
__global__ __launch_bounds__(64) void k_mlp_wgrad1(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dh1,
                                                   int n, MlpLayout lay, float *G, int chunk) {
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int col0 = blockIdx.x * 64;
  const long sA = (long)blockIdx.y * chunk, sB = min((long)n, sA + chunk);
  f32x4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (long s0 = sA; s0 < sB; s0 += 16) {
    bf16x4_t A[4], B[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long s = s0 + 4 * g + j;
        A[mt][j] = (short)(s < sB ? dh1[s * kHidden + 16 * mt + r] : 0);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = col0 + 16 * nt + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long s = s0 + 4 * g + j;
        B[nt][j] = (short)(s < sB && c < KP ? x[s * KP + c] : 0);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma16(A[mt], B[nt], acc[mt][nt]);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = col0 + 16 * nt + r;
      if (c < lay.F)
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(&G[(long)(16 * mt + 4 * g + i) * lay.F + c], acc[mt][nt][i]);
    }
}

// Adam on the fp32 master parameters; refreshes the bf16 copies and clears
// the gradient.  step >= 1; step == 0 only copies master -> bf16.
__global__ __launch_bounds__(kBlock) void k_mlp_adam(float *M, float *m1, float *m2, float *G, uint16_t *W,
                                                     MlpLayout lay, float lr, int step) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= lay.nmaster()) {  // zeros in the padding of W1P
    const long idx = k - lay.nmaster();
    if (idx >= lay.npad()) return;
    const int pad = lay.bv() - lay.fv();
    const int o = (int)(idx / (4 * pad)), v = (int)(idx / pad % 4), f = lay.fv() + (int)(idx % pad);
    W[lay.w1p_at(o, v, f)] = 0;
    return;
  }
  float w = M[k];
  if (step > 0) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gk = G[k];
    const float a = b1 * m1[k] + (1.f - b1) * gk;
    const float b = b2 * m2[k] + (1.f - b2) * gk * gk;
    m1[k] = a;
    m2[k] = b;
    const float ah = a / (1.f - powf(b1, (float)step));
    const float bh = b / (1.f - powf(b2, (float)step));
    w -= lr * ah / (sqrtf(bh) + eps);
    M[k] = w;
    G[k] = 0.f;
  }
  if (k < lay.mW2()) {
    const long o = k / lay.F, c = k % lay.F;
    W[lay.w1() + o * lay.KP + c] = f2bf(w);
    if (lay.has_w1p()) {
      const int v = (int)(c / lay.fv()), f = (int)(c % lay.fv());
      W[lay.w1p_at((int)o, v, f)] = f2bf(w);
    }
  } else if (k < lay.mw3()) {
    const long o = (k - lay.mW2()) / kHidden, c = (k - lay.mW2()) % kHidden;
    W[lay.w2() + o * kHidden + c] = f2bf(w);
    W[lay.w2t() + c * kHidden + o] = f2bf(w);
  } else if (k < lay.mb1()) {
    W[lay.w3() + (k - lay.mw3())] = f2bf(w);
  }
}

// ---------------------------------------------------------------------------
// The limiter's learned indicator (2D Euler): p > band_hi flags a cell,
// p < band_lo clears it, and the TVB decision settles the band in between.
// ---------------------------------------------------------------------------
struct LearnedArgs {
  const uint16_t *W;
  const float *M;
  MlpLayout lay;
  float band_lo, band_hi;
  float *prob;  // may be null: per-cell probability
};

// Work layout: a block of lm_waves(N) wavefronts shares the network's
// weights in LDS; each wavefront owns a strip of kLmStrip columns (lane
// slots 1..14 of its 16; slots 0 and 15 are the x-halo) and marches up a
// chunk of rows.  Lane (r, g) holds variable g of slot r.  The rows below,
// at and above the current one are kept in registers (one load per value),
// west and east neighbours come from the adjacent slots.  The network is
// evaluated transposed, H^T = W X^T, with the weights as the MFMA A operand:
// the B fragment of k-block kb held by lane (r, g) is features 4 kb .. 4 kb + 3
// of variable g of cell r, i.e. the lane's own features, so they go to the
// MFMA straight from registers; each layer's output fragments are the next
// layer's B fragments.
template <int N>
struct LmShape {
  static constexpr int NP = N + 1, NM = NP * NP, FV = 5 * NM, BV = (FV + 3) / 4 * 4;
  static constexpr int FK = BV % 8 == 0 ? 8 : 4, KB = BV / FK;  // features per lane and k-block (MlpLayout::frag)
  static constexpr int KP = 4 * BV;  // padded input width (= (F + 15) / 16 * 16 for F = 4 FV)
  static constexpr int W1 = kHidden * KP, W2 = kHidden * kHidden;
  static constexpr int W3 = kHidden;  // w3 in layer-3 fragment order [kb][g][e]
  static constexpr int PAR = 2 * (2 * kHidden + 2);  // b1 | b2 | b3 as floats (in bf16 slots)
  static constexpr int WAVES = lm_waves(N);
  static constexpr int LDS = W1 + W2 + W3 + PAR;
};

// Copies the weights into LDS in fragment order (whole block), then a barrier.
template <int N>
__device__ inline void lm_load_weights(const LearnedArgs &L, uint16_t *wl) {
  using S = LmShape<N>;
  const int tid = threadIdx.x, nt = blockDim.x;
  const uint16_t *__restrict__ W1P = L.W + L.lay.w1p();
  for (int k = tid; k < S::W1 / 4; k += nt)
    reinterpret_cast<uint2 *>(wl)[k] = reinterpret_cast<const uint2 *>(W1P)[k];
  // W2 A-fragments: element e of lane (r, g), k-block kb, output block nb is
  // W2[16 nb + r][c] with c = 16 kb + 4 g + e (K = 4), or, for K = 8, the
  // hidden units that lane's layer-1 output blocks 2 kb and 2 kb + 1 hold:
  // c = 16 (2 kb + e / 4) + 4 g + e % 4
  const uint16_t *__restrict__ W2 = L.W + L.lay.w2();
  for (int k = tid; k < S::W2; k += nt) {
    int e, ln, c, nb;
    if constexpr (S::FK == 8) {
      e = k & 7, ln = (k >> 3) & 63, nb = k >> 10;
      const int kb = (k >> 9) & 1;
      c = 16 * (2 * kb + e / 4) + 4 * (ln >> 4) + e % 4;
    } else {
      e = k & 3, ln = (k >> 2) & 63, nb = k >> 10;
      const int kb = (k >> 8) & 3;
      c = 16 * kb + 4 * (ln >> 4) + e;
    }
    wl[S::W1 + k] = W2[(16 * nb + (ln & 15)) * kHidden + c];
  }
  // w3 as the A fragment of layer 3 (every row of A the same): element e of
  // lane group g, k-block kb is w3[c] with c the hidden unit of element e of
  // that group's layer-2 B fragment (the column map of W2 above)
  for (int k = tid; k < S::W3; k += nt) {
    const int e = k % S::FK, gg = (k / S::FK) & 3, kb = k / (4 * S::FK);
    const int c = S::FK == 8 ? 16 * (2 * kb + e / 4) + 4 * gg + e % 4 : 16 * kb + 4 * gg + e;
    wl[S::W1 + S::W2 + k] = L.W[L.lay.w3() + c];
  }
  float *par = reinterpret_cast<float *>(wl + S::W1 + S::W2 + S::W3);
  for (int k = tid; k < kHidden; k += nt) {
    par[k] = L.M[L.lay.mb1() + k];
    par[kHidden + k] = L.M[L.lay.mb2() + k];
  }
  if (tid == 0) par[2 * kHidden] = L.M[L.lay.mb3()];
  __syncthreads();
}

// The value of lane r - 1 (UP) or r + 1 within each row of 16 lanes by a DPP
// row shift (a register move, no LDS round trip); the lane with no source in
// its row keeps its own value.  The shift writes a register other than its
// source.
template <bool UP>
__device__ __forceinline__ double row_shift1(double v) {
  constexpr int ctrl = UP ? 0x111 : 0x101;  // row_shr:1 / row_shl:1
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
  const int r = __lane_id() & 15;
  return (UP ? r == 0 : r == 15) ? v
                                 : __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The same shifts reading 0 in the lane with no source (the x-halo slots,
// whose results are never used): no select, and the f32 form folds into the
// DPP operand of the instruction that uses it.
template <bool UP>
__device__ __forceinline__ float row_shift0(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), UP ? 0x111 : 0x101, 0xF, 0xF, true));
}
template <bool UP>
__device__ __forceinline__ double row_shift0(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, UP ? 0x111 : 0x101, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), UP ? 0x111 : 0x101, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// max(x, 0) on the bit pattern: a negative float is a negative integer
// (one integer max, no NaN quieting of the MFMA results first)
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
// the larger of two non-negative floats, by their bit patterns
__device__ __forceinline__ float max_nonneg(float a, float b) {
  return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

typedef __bf16 bf16x2h_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// two floats to bf16 (nearest even) in one conversion
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2h_t));
}
__device__ __forceinline__ bf16x4_t pk4_bf16(float a, float b, float c, float d) {
  const uint2 v{pk_bf16(a, b), pk_bf16(c, d)};
  return __builtin_bit_cast(bf16x4_t, v);
}
__device__ __forceinline__ bf16x8_t cat8(bf16x4_t lo, bf16x4_t hi) {
  const uint2 a = __builtin_bit_cast(uint2, lo), b = __builtin_bit_cast(uint2, hi);
  return __builtin_bit_cast(bf16x8_t, uint4{a.x, a.y, b.x, b.y});
}
__device__ __forceinline__ bf16x8_t load8(const uint16_t *p) { return *reinterpret_cast<const bf16x8_t *>(p); }
// D += A B for 16 x 32 A and 32 x 16 B fragments (eight bf16 per lane each)
__device__ __forceinline__ f32x4_t mfma32(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One wavefront's strip: columns x0-1 .. x0+14 (owned x0 .. x0+13), rows
// j0 .. j1-1.  emit(active, flag, margin, p, cell) is called by every lane
// once per row (active: an owned cell, from lane group 0).
//
// Features are formed in FP32 from the FP64 state: the four mean
// differences (to the centre's mean) in FP64 and then rounded, the other
// modes rounded once per row they enter; the scale s is the FP32 rounding of
// the exact maximum (rounding is monotonic), and each feature is the FP32
// product with 1 / s, then rounded to BF16 for the network.
template <int N, bool BND, typename Emit>
__device__ inline void lm_strip(const double *__restrict__ u, const Geometry &g, int x0, int j0, int j1,
                                const LearnedArgs &L, const uint16_t *__restrict__ wl, Emit &&emit) {
  using S = LmShape<N>;
  constexpr int NP = S::NP, NM = S::NM, NH = NM - 1, FV = S::FV, KB = S::KB;
  const OrderTables &T = c_tab[N];
  const int lane = threadIdx.x & 63, r = lane & 15, gv = lane >> 4;
  int col = x0 + r - 1;
  if (col > g.nx) col = g.nx;
  const bool owner = r >= 1 && r <= kLmStrip && col < g.nx;
  const long plane = (long)g.nx * g.ny;
  const float *par = reinterpret_cast<const float *>(wl + S::W1 + S::W2 + S::W3);  // b1 | b2 | b3
  const double *__restrict__ up = u + (long)gv * NM * plane;
  // Row jj's modes of the lane's variable.  On periodic and transmissive
  // sides (!BND) a mirrored ghost's odd modes change sign: the loads are
  // issued here and the signs fixed by fix_row once the values are needed
  // (only where some lane of the wavefront holds such a ghost).
  struct Flip {
    bool fx, fy, any;
  };
  auto loadrow = [&](int jj, double (&R)[NM]) -> Flip {
    if (jj > g.ny) jj = g.ny;
    const CellIdx ci = map_cell<BND>(g, col, jj);
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      if constexpr (BND)
        R[q] = cell_mode<NP, NM, 2>(u, plane, g, ci, gv, q);
      else
        R[q] = up[(long)q * plane + ci.idx];
    }
    if constexpr (BND)
      return Flip{false, false, false};
    else
      return Flip{ci.fx, ci.fy, __any(ci.fx || ci.fy) != 0};
  };
  auto fix_row = [&](const Flip &f, double (&R)[NM]) {
    if (f.any) {
#pragma unroll
      for (int q = 0; q < NM; ++q) {
        const int m = q % NP, n = q / NP;
        if ((f.fx && (m & 1)) != (f.fy && (n & 1))) R[q] = -R[q];
      }
    }
  };
  // a row's modes but the mean in FP32; returns their largest magnitude
  auto to32 = [&](const double (&R)[NM], float (&F)[NH]) {
    float m = 0.f;
#pragma unroll
    for (int q = 1; q < NM; ++q) {
      F[q - 1] = (float)R[q];
      m = fmaxf(m, fabsf(F[q - 1]));
    }
    return m;
  };
  double Sm, Cv[NM], Nv[NM];  // Sm: the south neighbour's mean
  float S32[NH], C32[NH], N32[NH], hS, hC, hN;
  {
    double Sv[NM];
    fix_row(loadrow(j0 - 1, Sv), Sv);
    Sm = Sv[0];
    hS = to32(Sv, S32);
  }
  fix_row(loadrow(j0, Cv), Cv);
  fix_row(loadrow(j0 + 1, Nv), Nv);
  hC = to32(Cv, C32);
  hN = to32(Nv, N32);
  const float Mh2 = (float)g.tvb_Mx;
  const double k0 = T.b0[0] * T.b0[0];
  const f32x4_t *b1f = reinterpret_cast<const f32x4_t *>(par + 4 * gv);
  const f32x4_t *b2f = reinterpret_cast<const f32x4_t *>(par + kHidden + 4 * gv);
  // the layer-2 weight fragments are read from LDS per row (in registers they
  // would cost the third wavefront per SIMD at Q2)
  constexpr bool w2_regs = false;
  constexpr int FK = S::FK, KB2 = kHidden / (4 * FK);  // layer-2 k-blocks
  auto w2frag = [&](int nb, int kb) { return wl + S::W1 + ((nb * KB2 + kb) * 64 + lane) * FK; };
  bf16x4_t w2f[w2_regs ? 4 : 1][w2_regs ? 4 : 1];  // K = 8: [nb][2 kb + half]
  if constexpr (w2_regs) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        w2f[nb][kb] = FK == 8 ? load4(w2frag(nb, kb / 2) + 4 * (kb % 2)) : load4(w2frag(nb, kb));
  }
  for (int j = j0; j < j1; ++j) {
    double Pv[NM];
    const Flip fp = loadrow(j + 2, Pv);  // in flight while this row is evaluated
    // TVB decision of this variable (the expressions of tvb_cell), combined
    // over the cell's lanes; only needed for a probability inside the band
    auto tvb_decision = [&](bool &tflag, double &tmg) {
      tflag = false;
      tmg = INFINITY;
      const double mean = Cv[0] * k0;
#pragma unroll
      for (int dir = 0; dir < 2; ++dir) {
        const double Mh2 = dir == 0 ? g.tvb_Mx : g.tvb_My;
        const double mp = (dir == 0 ? row_shift1<false>(Cv[0]) : Nv[0]) * k0;
        const double mm = (dir == 0 ? row_shift1<true>(Cv[0]) : Sm) * k0;
        double upv = 0.0, umv = 0.0;
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          const int m = q % NP, n = q / NP;
          const double bu = dir == 0 ? T.bp[m] * T.b0[n] : T.b0[m] * T.bp[n];
          const double bd = dir == 0 ? T.bm[m] * T.b0[n] : T.b0[m] * T.bm[n];
          upv += Cv[q] * bu;
          umv += Cv[q] * bd;
        }
        const double dp = mp - mean, dm = mean - mm;
        tflag |= tvb_test(upv - mean, dp, dm, Mh2, tmg);
        tflag |= tvb_test(mean - umv, dp, dm, Mh2, tmg);
      }
      int fi = tflag ? 1 : 0;
      fi |= __shfl_xor(fi, 16);
      fi |= __shfl_xor(fi, 32);
      tflag = fi != 0;
      tmg = fmin(tmg, __shfl_xor(tmg, 16));
      tmg = fmin(tmg, __shfl_xor(tmg, 32));
    };
    // features of variable gv: C, W, E, S, N, each with its modes; the
    // means relative to the centre's (whose own entry is 0); scaled by 1 / s
    const double c0 = Cv[0];
    const float dW = (float)(row_shift0<true>(c0) - c0), dE = (float)(row_shift0<false>(c0) - c0);
    const float dS = (float)(Sm - c0), dN = (float)(Nv[0] - c0);
    float mx = max_nonneg(max_nonneg(Mh2, hC), max_nonneg(hS, hN));
    mx = max_nonneg(mx, max_nonneg(row_shift0<true>(hC), row_shift0<false>(hC)));
    mx = max_nonneg(mx, max_nonneg(max_nonneg(fabsf(dW), fabsf(dE)), max_nonneg(fabsf(dS), fabsf(dN))));
    const float inv = __builtin_amdgcn_rcpf(mx);
    auto feature = [&](int f) -> float {
      if (f >= FV) return 0.f;  // padding
      const int c = f / NM, q = f % NM;
      if (q == 0) return c == 0 ? 0.f : (c == 1 ? dW : (c == 2 ? dE : (c == 3 ? dS : dN))) * inv;
      switch (c) {
        case 0: return C32[q - 1] * inv;
        case 1: return row_shift0<true>(C32[q - 1]) * inv;
        case 2: return row_shift0<false>(C32[q - 1]) * inv;
        case 3: return S32[q - 1] * inv;
        default: return N32[q - 1] * inv;
      }
    };
    // layer 1: H1^T = W1 X^T (+ b1 as the accumulator's start)
    f32x4_t h[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) h[nb] = b1f[4 * nb];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int f = FK * kb;
      const bf16x4_t x = pk4_bf16(feature(f), feature(f + 1), feature(f + 2), feature(f + 3));
      if constexpr (FK == 8) {
        const bf16x8_t x8 = cat8(x, pk4_bf16(feature(f + 4), feature(f + 5), feature(f + 6), feature(f + 7)));
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) h[nb] = mfma32(load8(wl + ((nb * KB + kb) * 64 + lane) * 8), x8, h[nb]);
      } else {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) h[nb] = mfma16(load4(wl + ((nb * KB + kb) * 64 + lane) * 4), x, h[nb]);
      }
      __builtin_amdgcn_sched_barrier(0);  // keeps each k-block's fragment loads next to their use (registers)
    }
    bf16x4_t h1[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      h1[nb] = pk4_bf16(relu_bits(h[nb][0]), relu_bits(h[nb][1]), relu_bits(h[nb][2]), relu_bits(h[nb][3]));
    // layer 2: H2^T = W2 H1^T (+ b2); for K = 8 the B fragment of k-block kb
    // is the lane's layer-1 blocks 2 kb and 2 kb + 1
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) h[nb] = b2f[4 * nb];
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        if constexpr (FK == 8) {
          const bf16x8_t a = w2_regs ? cat8(w2f[w2_regs ? nb : 0][w2_regs ? 2 * kb : 0],
                                            w2f[w2_regs ? nb : 0][w2_regs ? 2 * kb + 1 : 0])
                                     : load8(w2frag(nb, kb));
          h[nb] = mfma32(a, cat8(h1[2 * kb], h1[2 * kb + 1]), h[nb]);
        } else {
          h[nb] = mfma16(w2_regs ? w2f[w2_regs ? nb : 0][w2_regs ? kb : 0] : load4(w2frag(nb, kb)), h1[kb], h[nb]);
        }
      }
    // layer 3 on the BF16-rounded activations, as one more MFMA layer: w3
    // is the A fragment with all 16 rows the same and b3 the accumulator's
    // start, so every element of the lane's result is its cell's logit
    bf16x4_t h2[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      h2[nb] = pk4_bf16(relu_bits(h[nb][0]), relu_bits(h[nb][1]), relu_bits(h[nb][2]), relu_bits(h[nb][3]));
    const float b3 = par[2 * kHidden];
    f32x4_t z{b3, b3, b3, b3};
    const uint16_t *w3f = wl + S::W1 + S::W2 + gv * FK;
    if constexpr (FK == 8) {
#pragma unroll
      for (int kb = 0; kb < KB2; ++kb) z = mfma32(load8(w3f + 32 * kb), cat8(h2[2 * kb], h2[2 * kb + 1]), z);
    } else {
#pragma unroll
      for (int kb = 0; kb < KB2; ++kb) z = mfma16(load4(w3f + 16 * kb), h2[kb], z);
    }
    const float p = __builtin_amdgcn_rcpf(1.f + __expf(-z[0]));
    bool flag = false;
    double mg = INFINITY;
    const bool in_band = !(p > L.band_hi) && !(p < L.band_lo);
    if (__any(in_band)) {  // the whole wavefront takes part (shuffles inside)
      bool tflag;
      double tmg;
      tvb_decision(tflag, tmg);
      if (in_band) {
        flag = tflag;
        mg = tmg;
      }
    }
    if (p > L.band_hi) flag = true;
    emit(owner && gv == 0, flag, mg, p, (long)j * g.nx + col);
    Sm = c0;
    fix_row(fp, Pv);
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      Cv[q] = Nv[q];
      Nv[q] = Pv[q];
    }
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      S32[q] = C32[q];
      C32[q] = N32[q];
    }
    hS = hC;
    hC = hN;
    hN = to32(Nv, N32);
  }
}

// The flagged cells of one wavefront's strip chunk, gathered in LDS and
// appended to a troubled list with one atomic at the end: one atomic per row
// and wavefront contends for the counter once most rows hold a troubled cell
// (a learned pass at t = 0.05 of the 2048^2 run took 1.5 ms that way).
template <typename E>
struct WaveList {
  static constexpr int kCap = kLmRows * 16;  // rows x lane slots of a chunk
  E *buf;  // LDS, kCap entries
  int n;   // entries so far (the same in every lane)
  __device__ void push(bool flag, E entry) {
    const unsigned long long ballot = __ballot(flag);
    if (flag) buf[n + __popcll(ballot & ((1ull << __lane_id()) - 1ull))] = entry;
    n += __popcll(ballot);
  }
  // reserve(k) (called by one lane) returns the list index of k new entries
  template <typename R>
  __device__ void flush(R &&reserve, E *list) {
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (n > 0) {
      if (__lane_id() == 0) base = reserve(n);
      base = __shfl(base, 0);
    }
    for (int k = __lane_id(); k < n; k += 64) list[base + k] = buf[k];
    n = 0;
    __builtin_amdgcn_wave_barrier();
  }
};

// Single mesh: grid (strip groups, row chunks of kLmRows); block = lm_waves(N) wavefronts.
template <int N, int EQ, bool BND>
__global__ __launch_bounds__(64 * lm_waves(N), lm_occupancy(N)) void k_indicator_learned(LimitArgs a, LearnedArgs L, int rows) {
  static_assert(EQ == 1, "learned indicator: 2D Euler");
  using S = LmShape<N>;
  __shared__ __align__(16) uint16_t lds[S::LDS];
  __shared__ int32_t flagged[S::WAVES][WaveList<int32_t>::kCap];
  if (a.check_done && a.sc->done) return;
  lm_load_weights<N>(L, lds);
  const Geometry &g = a.geo;
  const int wave = threadIdx.x >> 6;
  const int x0 = (blockIdx.x * S::WAVES + wave) * kLmStrip;
  if (x0 >= g.nx) return;  // no barrier follows
  const int j0 = blockIdx.y * rows, j1 = min(j0 + min(rows, kLmRows), g.ny);
  WaveList<int32_t> wl{flagged[wave], 0};
  lm_strip<N, BND>(a.u, g, x0, j0, j1, L, lds,
              [&](bool active, bool flag, double mg, float p, long cell) {
                if (active) {
                  if (L.prob) L.prob[cell] = p;
                  if (a.ovr) flag = a.ovr[cell] != 0;
                  if (a.flags) a.flags[cell] = flag ? 1 : 0;
                  if (a.margin) a.margin[cell] = mg;
                }
                wl.push(active && flag, (int32_t)cell);
              });
  wl.flush([&](int k) {
    atomicAdd(&a.sc->troubled_total, (unsigned long long)k);
    return atomicAdd(a.count, k);
  }, a.list);
}
