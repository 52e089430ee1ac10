// HIP loop kernel for gfx950 (CDNA4): the temperature-flow loops of the TUfRG
// right-hand side on the fine momentum grid.
//
// Driven by a table of work items (point, a, b, c) like every kernel of the
// library: one launch covers any set of points with uneven grids and
// truncations.  Temperatures are read from a per-point device array (so that a
// captured HIP graph can be replayed with new temperatures), and points whose
// flow has stopped are skipped through a per-point device flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "loop_body.h"
#include "transforms.h"
#include "tufrg_internal.h"

namespace tufrg {
namespace {

// Loop kernel over work items (p, q * nsplit + split); SMAX is the largest
// smax of the batch, and each item runs the body compiled for its own smax;
// OMEGA selects the regulator (Omega cutoff at T = 0, else temperature);
// UNROLL keeps two FP64 rows in flight (more registers, fewer blocks per CU).
// (A single-point form reading its tables from the launch's arguments, as
// the fused launch below does, ran slower here: 9.9 -> 10.2 us.)
// Without a queue every block runs item blockIdx.x (the hardware dispatcher
// balances the load, items being ordered costliest first); with a queue the
// kernel is persistent and blocks take items until the queue is empty.
template <int SMAX, bool MIXED, bool OMEGA, bool UNROLL>
__global__ void __launch_bounds__(kLoopThreadsMax)
k_loops(Batch b, const int4* __restrict__ items, int nitems, int* __restrict__ queue) {
  extern __shared__ double smem[];
  __shared__ int cur;
  if (b.item_count != nullptr) nitems = min(nitems, *b.item_count);
  if (queue == nullptr) {
    if ((int)blockIdx.x < nitems) loop_dispatch<SMAX, MIXED, OMEGA, UNROLL>(b, items[blockIdx.x], smem);
    return;
  }
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) cur = atomicAdd(queue, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= nitems) break;
    loop_dispatch<SMAX, MIXED, OMEGA, UNROLL>(b, items[it], smem);
  }
  if (t == 0 && atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
    atomicExch(queue, 0);
    atomicExch(queue + 1, 0);
  }
}

// The loops and the forward transform of the projections in one launch (they
// are independent: the loops read only the temperature, the transform only
// the couplings): blocks below nloop run loop items, the others forward-
// transform items, so that both fill the machine together without a second
// stream.  Dynamic shared memory holds the larger of the two layouts.  ONE:
// a single-point launch (compiled for the point's own smax; its tables come
// from the launch's arguments, one dependent load fewer per block).
template <int SMAX, bool MIXED, int KT, bool OMEGA, bool ONE>
__global__ void __launch_bounds__(kLoopThreadsMax)
k_loops_fwd(Batch b, const int4* __restrict__ loop_items, int nloop, const int4* __restrict__ fwd_items,
            const double* __restrict__ X, TArg ta) {
  extern __shared__ double smem[];
  if (blockIdx.x == 0) {
    // the temperatures, stored for the kernels after this launch (the loop
    // blocks of this launch take them from ta)
    if (ta.mode == 1) {
      for (int i = threadIdx.x; i < ta.n; i += blockDim.x) ta.Tp[ta.p0 + i] = ta.v[i];
    } else if (ta.mode == 2) {
      const double T = ta.Ttab[4 * ta.step[0] + ta.stage];
      for (int i = threadIdx.x; i < ta.npts; i += blockDim.x) ta.Tp[i] = T;
    } else if (ta.mode == 3) {
      for (int i = threadIdx.x; i < ta.npts; i += blockDim.x) ta.Tp[i] = exp(fma(ta.c, ta.h[i], ta.s[i]));
    }
  }
  if ((int)blockIdx.x < nloop) {
    loop_dispatch<SMAX, MIXED, OMEGA, true, ONE>(b, loop_items[blockIdx.x], smem, &ta);
    return;
  }
  const int4 item = fwd_items[blockIdx.x - nloop];
  const int p = ONE ? 0 : item.x;
  if (skip_point(b, p)) return;
  if constexpr (MIXED) fwd_mix_body<KT>(b, point_tables<ONE>(b, p), item, X, smem);
  else fwd_part_body<KT>(b, point_tables<ONE>(b, p), item, X, smem);
}

// Calls f(smax, mixed, omega) with the runtime values as compile-time constants.
template <class F>
void with_loop_variant(int smax_max, bool mixed, bool omega, F&& f) {
  auto by_reg = [&](auto sm, auto mx) {
    if (omega) f(sm, mx, std::true_type{});
    else f(sm, mx, std::false_type{});
  };
  auto by_prec = [&](auto sm) {
    if (mixed) by_reg(sm, std::true_type{});
    else by_reg(sm, std::false_type{});
  };
  switch (smax_max) {
    case 0: by_prec(std::integral_constant<int, 0>{}); break;
    case 2: by_prec(std::integral_constant<int, 2>{}); break;
    default: by_prec(std::integral_constant<int, 4>{}); break;
  }
}

}  // namespace

void launch_loops(const Launch& L, const ItemRange& r, int* queue, bool mixed, hipStream_t s) {
  if (r.n <= 0) return;
  if (!L.loop_persistent) queue = nullptr;
  const int grid = L.loop_persistent ? std::min(r.n, L.loop_blocks) : r.n;
  const dim3 blk(L.loop_threads);
  const size_t sm = L.loop_smem;
  const int4* it = L.loop_items + r.begin;
  with_loop_variant(L.smax_max, mixed, L.omega, [&](auto S, auto M, auto O) {
    constexpr int SM = decltype(S)::value;
    constexpr bool MX = decltype(M)::value, OM = decltype(O)::value;
    if (L.loop_unroll)
      hipLaunchKernelGGL((k_loops<SM, MX, OM, true>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
    else
      hipLaunchKernelGGL((k_loops<SM, MX, OM, false>), dim3(grid), blk, sm, s, L.b, it, r.n, queue);
  });
}

void launch_loops_fwd(const Launch& L, const Ranges& r, const double* X, bool mixed, bool cross,
                      const TArg& ta, hipStream_t s) {
  const int nf = cross ? r.fwd.n : 0;
  if (r.loop.n + nf <= 0) return;
  const dim3 g(r.loop.n + nf), blk(L.front_threads);
  const size_t sm = L.front_smem;
  const int4* li = L.loop_items + r.loop.begin;
  const int4* fi = L.fwd_items + r.fwd.begin;
  with_loop_variant(L.smax_max, mixed, L.omega, [&](auto S, auto M, auto O) {
    constexpr int SM = decltype(S)::value;
    constexpr bool MX = decltype(M)::value, OM = decltype(O)::value;
    auto go = [&](auto one) {
      constexpr bool ON = decltype(one)::value;
      switch (L.fwd_kt) {
        case 1: hipLaunchKernelGGL((k_loops_fwd<SM, MX, 1, OM, ON>), g, blk, sm, s, L.b, li, r.loop.n, fi, X, ta);
          break;
        case 2: hipLaunchKernelGGL((k_loops_fwd<SM, MX, 2, OM, ON>), g, blk, sm, s, L.b, li, r.loop.n, fi, X, ta);
          break;
        case 3: hipLaunchKernelGGL((k_loops_fwd<SM, MX, 3, OM, ON>), g, blk, sm, s, L.b, li, r.loop.n, fi, X, ta);
          break;
        default: hipLaunchKernelGGL((k_loops_fwd<SM, MX, 5, OM, ON>), g, blk, sm, s, L.b, li, r.loop.n, fi, X, ta);
          break;
      }
    };
    if (L.one_point) go(std::true_type{});
    else go(std::false_type{});
  });
}

const void* loop_kernel_symbol(int smax_max, bool mixed, bool omega, bool unroll) {
  const void* k = nullptr;
  with_loop_variant(smax_max, mixed, omega, [&](auto S, auto M, auto O) {
    constexpr int SM = decltype(S)::value;
    constexpr bool MX = decltype(M)::value, OM = decltype(O)::value;
    k = unroll ? (const void*)k_loops<SM, MX, OM, true> : (const void*)k_loops<SM, MX, OM, false>;
  });
  return k;
}

}  // namespace tufrg
