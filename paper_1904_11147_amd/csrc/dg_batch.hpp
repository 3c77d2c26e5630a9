// Batched execution of many independent 2D Euler meshes (sizes and orders
// mixed, each with its own CFL time step).  Included by the kernel
// translation unit inside its anonymous namespace.
//
// Per order N there is one work queue over the instances still advancing:
// their ids with inclusive prefix sums of stage tiles and of 64-cell row
// segments.  A single block rebuilds all queues after every time-step
// decision, so finished instances drop out without a host round trip and
// the whole step can be replayed from a captured graph.  The stage kernel
// takes one tile per wavefront on a grid of the order's full tile count
// (wavefronts past the live queue exit at once; a grid-stride loop here costs
// registers the tile body needs).  The indicator, reconstruction and scatter
// kernels are persistent: a fixed grid walks the queue with a grid-stride
// loop.  Work items find their instance by binary search.  Every cell is
// computed by the same device functions as in the single-mesh kernels, so a
// batched run reproduces single-mesh runs bit for bit.

// First queue entry k with end[k] > w (w below end[n-1]).
__device__ inline int queue_find(const int32_t *__restrict__ end, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (end[mid] > w) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// finalize != 0: every instance decides its next time step (an instance that
// met a non-physical state stops).  Then one wavefront per order rebuilds
// that order's queue with wavefront prefix sums.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void k_batch_decide(BatchInst *__restrict__ inst, int n,
                                                       BatchQueue *__restrict__ queue, int32_t *active,
                                                       int finalize) {
  const int tid = threadIdx.x;
  if (tid == 0) *active = 0;
  if (finalize) {
    for (int i = tid; i < n; i += blockDim.x) {
      DevScalars *sc = inst[i].sc;
      if (sc->status) sc->done = 1;
      decide_dt(sc, 2, inst[i].cfl, inst[i].geo.hx, inst[i].geo.hy);
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  if (wave < 1 || wave > kMaxN) return;
  const int order = wave;
  BatchQueue &q = queue[order];
  int base = 0, tiles = 0, segs = 0, ltiles = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    int ca = 0, ct = 0, cs = 0, cl = 0;
    if (i < n) {
      const BatchInst &I = inst[i];
      if (I.order == order && !I.sc->done) {
        ca = 1;
        ct = I.tiles_x * I.tiles_y;
        cs = I.segs;
        cl = I.ltiles;
      }
    }
    const bool act = ca != 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int a = __shfl_up(ca, o), b = __shfl_up(ct, o), c = __shfl_up(cs, o), d = __shfl_up(cl, o);
      if (lane >= o) {
        ca += a;
        ct += b;
        cs += c;
        cl += d;
      }
    }
    if (act) {
      const int k = base + ca - 1;
      q.inst[k] = i;
      q.tile_end[k] = tiles + ct;
      q.seg_end[k] = segs + cs;
      q.ltile_end[k] = ltiles + cl;
    }
    base += __shfl(ca, 63);
    tiles += __shfl(ct, 63);
    segs += __shfl(cs, 63);
    ltiles += __shfl(cl, 63);
  }
  if (lane == 0) {
    q.n_active = base;
    q.total_tiles = tiles;
    q.total_segs = segs;
    q.total_ltiles = ltiles;
    q.count[0] = q.count[1] = q.count[2] = q.count[3] = 0;
    atomicAdd(active, base);
  }
}

// Position of a row-segment work item: instance, row j and first column i0.
struct SegItem {
  int id, j, i0;
};

__device__ inline SegItem seg_item(const BatchInst *__restrict__ inst, const BatchQueue *__restrict__ q, int w) {
  const int k = queue_find(q->seg_end, q->n_active, w);
  SegItem s;
  s.id = q->inst[k];
  const int local = w - (k ? q->seg_end[k - 1] : 0);
  const int per_row = (inst[s.id].geo.nx + 63) / 64;
  s.j = local / per_row;
  s.i0 = (local % per_row) * 64;
  return s;
}

// Spectral radius of the cell means of every queued instance (first step of a
// call).
template <int N>
__global__ __launch_bounds__(64) void k_batch_speed(const BatchInst *__restrict__ inst,
                                                    const BatchQueue *__restrict__ q) {
  constexpr int NM = (N + 1) * (N + 1);
  using P = Phys<1, 2>;
  const OrderTables &T = c_tab[N];
  const int total = q->total_segs;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const SegItem s = seg_item(inst, q, w);
    const BatchInst &I = inst[s.id];
    const Geometry &g = I.geo;
    const int i = s.i0 + threadIdx.x;
    double sx = 0.0, sy = 0.0;
    bool bad = false;
    if (i < g.nx) {
      const long plane = (long)g.nx * g.ny, cell = (long)s.j * g.nx + i;
      const double k0 = T.b0[0] * T.b0[0];
      double m[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) m[v] = I.u[(long)(v * NM) * plane + cell] * k0;
      sx = P::template speed<0>(m, g.gamma, bad);
      sy = P::template speed<1>(m, g.gamma, bad);
    }
    if (bad) atomicOr(&I.sc->status, 1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sx = fmax(sx, __shfl_xor(sx, o));
      sy = fmax(sy, __shfl_xor(sy, o));
    }
    if (threadIdx.x == 0) {
      atomicMax(&I.sc->smax[0], (unsigned long long)__double_as_longlong(sx));
      atomicMax(&I.sc->smax[1], (unsigned long long)__double_as_longlong(sy));
    }
  }
}

// SSP-RK3 stage over the queued tiles of one order.  Stage 1: u -> A, 2: (A,
// u) -> B, 3: (B, u) -> u; stage 0 writes the residual of u into A.
// Batches take periodic and transmissive sides only (checked on the host).
template <int N, int STAGE>
__global__ __launch_bounds__(64, 2) void k_batch_stage(const BatchInst *__restrict__ inst,
                                                       const BatchQueue *__restrict__ q) {
  __shared__ double row[euler_vpl(N) * (N + 1) * (N + 1) * 64];
  const int total = q->total_tiles;
  if ((int)blockIdx.x >= total) return;
  const int w = xcd_tile(blockIdx.x, total);
  const int k = queue_find(q->tile_end, q->n_active, w);
  const BatchInst &I = inst[q->inst[k]];
  const int local = w - (k ? q->tile_end[k - 1] : 0);
  StageArgs a;
  a.u = STAGE <= 1 ? I.u : (STAGE == 2 ? I.A : I.B);
  a.un = I.u;
  a.out = STAGE <= 1 ? I.A : (STAGE == 2 ? I.B : I.u);
  a.sc = I.sc;
  a.geo = I.geo;
  a.want_speed = 1;
  euler_tile<N, STAGE, false, true>(a, local % I.tiles_x, local / I.tiles_x, I.rows, row);
}

// Buffers of the limiter pass after stage SLOT+1: the state it limits and the
// side buffer that receives the reconstructed modes.
template <int SLOT>
__device__ inline double *limit_target(const BatchInst &I) {
  return SLOT == 0 ? I.A : (SLOT == 1 ? I.B : I.u);
}
template <int SLOT>
__device__ inline double *limit_side(const BatchInst &I) {
  return SLOT == 0 ? I.B : I.A;
}

// Troubled-cell indicator over the queued row segments (one wavefront per
// segment).  IND: DG_IND_TVB, DG_IND_ALL or DG_IND_KXRCF.
// The flagged cells of a wavefront's segments are gathered in LDS and
// appended to the order's list with one atomic per few segments (WaveList).
template <int N, int SLOT, int IND>
__global__ __launch_bounds__(64) void k_batch_indicator(const BatchInst *__restrict__ inst, BatchQueue *q,
                                                        long long *__restrict__ list) {
  __shared__ long long flagged[WaveList<long long>::kCap];
  WaveList<long long> wl{flagged, 0};
  auto reserve = [&](int k) { return atomicAdd(&q->count[SLOT], k); };
  const int total = q->total_segs;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const SegItem s = seg_item(inst, q, w);
    const BatchInst &I = inst[s.id];
    const Geometry &g = I.geo;
    const int i = s.i0 + threadIdx.x;
    bool flag = false;
    double mg = INFINITY;
    if (i < g.nx)
      flag = IND == DG_IND_ALL     ? true
             : IND == DG_IND_KXRCF ? kxrcf_cell<N, 1, 2, false>(limit_target<SLOT>(I), g, i, s.j, mg)
                                   : tvb_cell<N, 1, 2, false>(limit_target<SLOT>(I), g, i, s.j, mg);
    const long long cell = (long long)s.j * g.nx + i;
    const unsigned long long ballot = __ballot(flag);
    if (ballot && __lane_id() == 0) atomicAdd(&I.sc->troubled_total, (unsigned long long)__popcll(ballot));
    wl.push(flag, ((long long)s.id << 32) | cell);
    if (wl.n > WaveList<long long>::kCap - 64) wl.flush(reserve, list);
  }
  wl.flush(reserve, list);
}

// Positivity-preserving scaling of the limited state over the queued row
// segments (one wavefront per segment); a non-admissible mean stops that
// instance (its status word).
template <int N, int SLOT>
__global__ __launch_bounds__(64) void k_batch_positivity(const BatchInst *__restrict__ inst,
                                                         const BatchQueue *__restrict__ q) {
  const int total = q->total_segs;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const SegItem s = seg_item(inst, q, w);
    const BatchInst &I = inst[s.id];
    const int i = s.i0 + threadIdx.x;
    if (i < I.geo.nx &&
        positivity_cell<N, 2>(limit_target<SLOT>(I), (long)I.geo.nx * I.geo.ny, (long)s.j * I.geo.nx + i, I.geo))
      atomicOr(&I.sc->status, 1);
  }
}

// The learned indicator over the queued learned tiles (lm_waves(N) strips of
// kLmRows rows each); the block keeps the order's network in LDS.
template <int N, int SLOT>
__global__ __launch_bounds__(64 * lm_waves(N), lm_occupancy(N)) void k_batch_learned(const BatchInst *__restrict__ inst, BatchQueue *q,
                                                                    long long *__restrict__ list, BatchLearned BL) {
  using S = LmShape<N>;
  __shared__ __align__(16) uint16_t lds[S::LDS];
  __shared__ long long flagged[S::WAVES][WaveList<long long>::kCap];
  const LearnedArgs L{BL.W, BL.M, MlpLayout{4 * S::FV, S::KP}, BL.band_lo, BL.band_hi, nullptr};
  lm_load_weights<N>(L, lds);
  const int wave = threadIdx.x >> 6;
  WaveList<long long> wl{flagged[wave], 0};
  const int total = q->total_ltiles;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int k = queue_find(q->ltile_end, q->n_active, w);
    const int id = q->inst[k];
    const BatchInst &I = inst[id];
    const Geometry &g = I.geo;
    const int local = w - (k ? q->ltile_end[k - 1] : 0);
    const int groups = ((g.nx + kLmStrip - 1) / kLmStrip + S::WAVES - 1) / S::WAVES;
    const int x0 = ((local % groups) * S::WAVES + wave) * kLmStrip;
    const int j0 = (local / groups) * kLmRows, j1 = min(j0 + kLmRows, g.ny);
    if (x0 >= g.nx) continue;  // no barrier in the loop
    lm_strip<N, false>(limit_target<SLOT>(I), g, x0, j0, j1, L, lds,
                [&](bool active, bool flag, double, float p, long cell) {
                  if (active && I.prob) I.prob[cell] = p;
                  wl.push(active && flag, ((long long)id << 32) | cell);
                });
    wl.flush([&](int k) {
      atomicAdd(&I.sc->troubled_total, (unsigned long long)k);
      return atomicAdd(&q->count[SLOT], k);
    }, list);
  }
}

template <int N, int SLOT>
__global__ __launch_bounds__(kBlock) void k_batch_csweno(const BatchInst *__restrict__ inst,
                                                         const BatchQueue *__restrict__ q,
                                                         const long long *__restrict__ list) {
  const long count = q->count[SLOT], total = count * 4;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long long e = list[t % count];  // one variable of consecutive entries per wavefront
    const BatchInst &I = inst[(int)(e >> 32)];
    csweno_cell<N, 1, 2, false>(limit_target<SLOT>(I), limit_side<SLOT>(I), I.geo, (long)(e & 0xffffffffll),
                                (int)(t / count));
  }
}

template <int N, int SLOT>
__global__ __launch_bounds__(kBlock) void k_batch_csweno_char(const BatchInst *__restrict__ inst,
                                                              const BatchQueue *__restrict__ q,
                                                              const long long *__restrict__ list) {
  const long total = q->count[SLOT];
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long long e = list[t];
    const BatchInst &I = inst[(int)(e >> 32)];
    csweno_char_cell<N, 2, false>(limit_target<SLOT>(I), limit_side<SLOT>(I), I.geo, (long)(e & 0xffffffffll));
  }
}

template <int N, int SLOT>
__global__ __launch_bounds__(kBlock) void k_batch_scatter(const BatchInst *__restrict__ inst,
                                                          const BatchQueue *__restrict__ q,
                                                          const long long *__restrict__ list) {
  constexpr int NM = (N + 1) * (N + 1), NV = 4;
  const long count = q->count[SLOT], total = count * NV * (NM - 1);
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / count;  // consecutive threads: consecutive entries of one plane
    const int m = 1 + (int)(r % (NM - 1));
    const int v = (int)(r / (NM - 1));
    const long long e = list[t % count];
    const BatchInst &I = inst[(int)(e >> 32)];
    const long plane = (long)I.geo.nx * I.geo.ny;
    const long k = (long)(v * NM + m) * plane + (long)(e & 0xffffffffll);
    limit_target<SLOT>(I)[k] = limit_side<SLOT>(I)[k];
  }
}
