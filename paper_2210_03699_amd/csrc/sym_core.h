// Work-item body of the symmetric pair sum, shared by the float64 and the
// mixed-precision kernels (each translation unit instantiates it with its
// own arithmetic policy).  The schedule is described in symmetric.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "operator.h"
#include "symmetric.h"

namespace ibim {
namespace sym {

constexpr int kT = kPairTile;
// The staged column tile is held as four sub-blocks of 64 sources, each
// followed by copies of its first kWrap sources, so that a lane sweeping a
// sub-block from a rotated start reads kWrap consecutive slots from one base
// address (LDS immediate offsets) without wrapping; the column sums have the
// same layout, and the sums in the copies are folded back at the end.
constexpr int kWrap = 8;
constexpr int kSlot = 64 + kWrap;  // slots per sub-block
constexpr int kSlots = 4 * kSlot;  // slots per staged tile

// Items of up to this many row tiles keep their row sums in LDS between
// column tiles; larger items carry them in their scratch slots.
constexpr int kLdsRows = 4;

// LDS slot of source j of the staged tile.
__device__ __forceinline__ int slot(int j) { return (j >> 6) * kSlot + (j & 63); }

__device__ __forceinline__ bool careful_pair(const SymArgs& a, int I, int J) {
  const int64_t bit = (int64_t)I * a.T + J;
  return (a.careful[bit >> 5] >> (bit & 31)) & 1u;
}

template <class T>
__device__ __forceinline__ T* lds_at(T* base, unsigned byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

template <class L>
struct SharedL {
  L rec;                                   // records of the column tile J
  // column sums of J (row 1, row 2) in two arrays of doubles: lanes add to
  // consecutive slots, 8 bytes apart, which keeps the LDS atomics free of
  // bank conflicts (a 16-byte stride gave 4-way conflicts)
  double cacc1[kSlots], cacc2[kSlots];
  // row sums of items of at most kLdsRows row tiles, lane-private
  double racc1[kLdsRows][kT], racc2[kLdsRows][kT];
};
// LDS of a policy P (policies with one record layout share one type)
template <class P>
using Shared = SharedL<typename P::Lds>;

// Sums over the sources of tile Y for the target of this lane in tile X
// (k = X*256 + tid), pairs of N_k skipped.  src(j) returns source j of Y.
template <class P, class Src>
__device__ __forceinline__ void one_way(const SymArgs& a, const typename P::Consts& pc, int X,
                                        int Y, const Src& src, double& S1, double& S2) {
  const int tid = threadIdx.x;
  const int32_t M = a.M;
  const int32_t k = X * kT + tid;
  const int32_t kc = k < M ? k : M - 1;
  const typename P::Rec t = P::load(a, kc);
  const int32_t s0 = Y * kT;
  const int n = min(kT, M - s0);
  int32_t p = a.crow[kc];
  const int32_t pe = a.crow[kc + 1];
  while (p < pe && a.ccol[p] < s0) ++p;
  int32_t nxt = p < pe ? a.ccol[p] : INT_MAX;
  for (int j = 0; j < n; ++j) {
    double d1, d2;
    P::one(t, src(j), pc, d1, d2);
    const bool ex = (s0 + j == nxt);
    if (ex) {
      ++p;
      nxt = p < pe ? a.ccol[p] : INT_MAX;
    }
    S1 += ex ? 0.0 : d1;
    S2 += ex ? 0.0 : d2;
  }
}

// The shared evaluations of NR row tiles (this lane's targets f[r]) against
// the staged column tile: four phases, wave w on sub-block (w + p) mod 4 in
// phase p, each lane sweeping the 64 sources from a rotated start, kWrap at a
// time from consecutive slots.  Row sums stay in S1, S2; the column sums of
// all NR targets for one source go to its slot with one LDS atomic.
template <class P, int NR>
__device__ __forceinline__ void sweep(Shared<P>& sh, const typename P::Consts& pc,
                                      const typename P::Rec (&f)[NR], double (&S1)[NR],
                                      double (&S2)[NR]) {
  const int tid = threadIdx.x;
  const int wv = tid >> 6, l = tid & 63;
  for (int ph = 0; ph < 4; ++ph) {
    // byte offset of sub-block (wv + ph) mod 4 in the 16-byte-record arrays
    const unsigned sb16 = (unsigned)(((wv + ph) & 3) * kSlot) << 4;
#pragma unroll 1
    for (int s0 = 0; s0 < 64; s0 += kWrap) {
      // this lane takes sources (l + s0 + k) mod 64, k < kWrap, from
      // consecutive slots (the copies after the sub-block cover the wrap)
      const unsigned off = ((((unsigned)l + (unsigned)s0) & 63u) << 4) + sb16;
      const unsigned off8 = off >> 1;  // the same slot in an array of doubles
#pragma unroll
      for (int k = 0; k < kWrap; ++k) {
        const typename P::Rec m = P::at(sh.rec, off + 16u * k);
        double C1, C2;
        P::template both<false>(f[0], m, pc, S1[0], S2[0], C1, C2);
#pragma unroll
        for (int r = 1; r < NR; ++r) P::template both<true>(f[r], m, pc, S1[r], S2[r], C1, C2);
        atomicAdd(lds_at(sh.cacc1, off8 + 8u * k), C1);
        atomicAdd(lds_at(sh.cacc2, off8 + 8u * k), C2);
      }
    }
    __syncthreads();
  }
}

// One work item (rb, cb).  Called by all 256 threads of the workgroup.
// The row sums of row tile I start at zero at the first column tile that
// meets I (J = max(J0, I)) and are carried to the next one in LDS (items of
// at most kLdsRows row tiles) or in the tile's (cb, I) slot of the row
// partial sums, read and written back by the thread that owns the row; the
// slot receives them scaled by h^3/(4 pi) at the last visit (J = J1 - 1),
// the second row by P::scale2 (h^3/(4 pi) times the policy's unit factor).
template <class P>
__device__ void item(const SymArgs& a, int rb, int cb, Shared<P>& sh) {
  double* const cacc1 = sh.cacc1;
  double* const cacc2 = sh.cacc2;
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int T = a.T;
  const int32_t M = a.M;
  const int rows = a.rows;
  const int I0 = rb * rows;
  const int J0 = cb * a.b, J1 = min(J0 + a.b, T);
  const int nCB = (T + a.b - 1) / a.b;
  const bool in_lds = rows <= kLdsRows;  // uniform
  const typename P::Consts pc = P::consts(a);
  auto row_sums = [&](int I) { return a.rowpart + sym_row_slot(cb, I, a.b, nCB) * (2 * kT); };
  auto row_load = [&](int i, int J, double& S1, double& S2) {
    const int I = I0 + i;
    if (J == max(J0, I)) {
      S1 = S2 = 0.0;
    } else if (in_lds) {
      S1 = sh.racc1[i][tid];
      S2 = sh.racc2[i][tid];
    } else {
      const double* rp = row_sums(I);
      S1 = rp[tid];
      S2 = rp[kT + tid];
    }
  };
  auto row_store = [&](int i, int J, double S1, double S2) {
    const int I = I0 + i;
    const bool last = J == J1 - 1;
    if (in_lds) {
      sh.racc1[i][tid] = S1;
      sh.racc2[i][tid] = S2;
    }
    if (last || !in_lds) {
      double* rp = row_sums(I);
      rp[tid] = (last ? a.scale : 1.0) * S1;
      rp[kT + tid] = (last ? P::scale2(a) : 1.0) * S2;
    }
  };

  for (int J = max(J0, I0); J < J1; ++J) {
    const int my = slot(tid);
    const bool wraps = l < kWrap;  // this source also has a copy after its sub-block
    {
      const int32_t m = J * kT + tid;
      if (m < M) {
        const typename P::Rec r = P::load(a, m);
        P::store(sh.rec, my, r);
        if (wraps) P::store(sh.rec, my + 64, r);
      }
      cacc1[my] = cacc2[my] = 0.0;
      if (wraps) cacc1[my + 64] = cacc2[my + 64] = 0.0;
    }
    __syncthreads();
    auto slow = [&](int I) {
      return I == J || careful_pair(a, I, J) || (J == T - 1 && M % kT != 0);
    };
    for (int i = 0; i < rows;) {
      const int I = I0 + i;
      if (I >= T || I > J) break;  // uniform; so are the later row tiles
      if (!slow(I) && i + 1 < rows && I + 1 < J && !slow(I + 1)) {
        // two row tiles against the staged sources: one LDS read and one
        // column-sum atomic serve two evaluations
        const typename P::Rec f[2] = {P::load(a, I * kT + tid), P::load(a, (I + 1) * kT + tid)};
        double S1[2], S2[2];
        row_load(i, J, S1[0], S2[0]);
        row_load(i + 1, J, S1[1], S2[1]);
        sweep<P, 2>(sh, pc, f, S1, S2);
        row_store(i, J, S1[0], S2[0]);
        row_store(i + 1, J, S1[1], S2[1]);
        i += 2;
        continue;
      }
      if (slow(I)) {
        double S1, S2;
        row_load(i, J, S1, S2);
        // row I from the sources of J (LDS broadcasts)
        one_way<P>(a, pc, I, J, [&](int j) { return P::at(sh.rec, (unsigned)slot(j) << 4); }, S1,
                   S2);
        row_store(i, J, S1, S2);
        if (I != J) {
          // row J from the sources of I (uniform global loads)
          double c1 = 0.0, c2 = 0.0;
          one_way<P>(a, pc, J, I, [&](int j) { return P::load(a, I * kT + j); }, c1, c2);
          cacc1[my] += c1;
          cacc2[my] += c2;
        }
        __syncthreads();
        ++i;
        continue;
      }
      const typename P::Rec f[1] = {P::load(a, I * kT + tid)};
      double S1[1], S2[1];
      row_load(i, J, S1[0], S2[0]);
      sweep<P, 1>(sh, pc, f, S1, S2);
      row_store(i, J, S1[0], S2[0]);
      ++i;
    }
    // column sums of J (this thread's slot and, for the first kWrap sources
    // of a sub-block, the copy slot; every add to them has completed)
    if (wraps) {
      cacc1[my] += cacc1[my + 64];
      cacc2[my] += cacc2[my + 64];
    }
    double* cp = a.colpart + sym_col_slot(rb, J, rows) * (2 * kT);
    cp[tid] = a.scale * cacc1[my];
    cp[kT + tid] = P::scale2(a) * cacc2[my];
    __syncthreads();  // LDS is refilled for the next column tile
  }
}

// Persistent loop over (problem, item) entries taken from *counter; body(a,
// rb, cb) runs one item with all threads of the workgroup.
template <class Body>
__device__ void batched(const SymArgs* __restrict__ probs, const int32_t* __restrict__ work,
                        int n_work, int* counter, const Body& body) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    // the entry index is uniform: keep it (and so the argument record) scalar
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // every thread has read `next` before it is overwritten
    if (it >= n_work) break;
    const int pi = __builtin_amdgcn_readfirstlane(work[2 * it]);
    const int ii = __builtin_amdgcn_readfirstlane(work[2 * it + 1]);
    const SymArgs a = probs[pi];
    const int2 it2 = a.items[ii];
    body(a, __builtin_amdgcn_readfirstlane(it2.x), __builtin_amdgcn_readfirstlane(it2.y));
    __syncthreads();  // LDS is reused by the next entry
  }
}

}  // namespace sym
}  // namespace ibim
