// Segment-per-cell dense LU: one small block per SEG-lane segment of a
// wavefront, lane r of the segment owns row r of the block in registers.
//
// Right-looking partial pivoting with LAPACK getrf semantics (first maximal
// pivot, whole-row exchange, division by the pivot).  Rows never move
// between lanes: every lane tracks the position its row holds in the
// permuted matrix, so an exchange of rows k and p swaps two position labels.
// The pivot search is a segmented arg-max over shuffles (ties go to the
// smaller current position, i.e. LAPACK's first maximum); the pivot row is
// published once through LDS and read back by the segment.
//
// Register indexing stays static without unrolling the whole elimination:
// the k loop runs in chunks of CH columns, and after every chunk each lane
// rotates its row left by CH, so inside a chunk the current column is always
// row[kk] for a compile-time kk.  After SEG/CH rotations the row is back in
// column order.  Blocks smaller than SEG are padded with identity rows and
// columns, which leaves the leading factors, pivots and solution exactly
// those of the unpadded block.
#pragma once

#include <hip/hip_runtime.h>

namespace bdfgpu {

template <int NP>
struct SegOf {
  static constexpr int value = NP <= 2 ? 2 : NP <= 4 ? 4 : NP <= 8 ? 8 : NP <= 16 ? 16 : NP <= 32 ? 32 : 64;
};

template <typename T>
__device__ __forceinline__ T sabs(T v) { return v < T(0) ? -v : v; }

// The value x holds in the lane paired with this one at level L of a
// butterfly over aligned groups of lanes: L = 0 and 1 pair lanes i ^ 1 and
// i ^ 2 (DPP quad permutes), L = 2 and 3 mirror 8- and 16-lane groups
// (i <-> 7 - i, i <-> 15 - i), L = 4 and 5 pair i ^ 16 and i ^ 32
// (v_permlane16/32_swap).  All are VALU lane moves, without the LDS-crossbar
// round trip of a shuffle.  After levels 0..L, a commutative and associative
// combine has reduced every aligned group of 2^(L+1) lanes, and every lane of
// the group holds the same bits.  The lanes of a group must be active.
template <int L>
__device__ __forceinline__ int lane_pair(int x) {
  if constexpr (L == 0) {
    return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  } else if constexpr (L == 1) {
    return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  } else if constexpr (L == 2) {
    return __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);   // row_half_mirror
  } else if constexpr (L == 3) {
    return __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false);   // row_mirror
  } else if constexpr (L == 4) {
    // [0]: the even 16-lane rows' values in every row, [1]: the odd rows'
    const auto e = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (threadIdx.x & 16) ? e[0] : e[1];
  } else {
    // [0]: the lower 32 lanes' values in both halves, [1]: the upper ones'
    const auto e = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x & 32) ? e[0] : e[1];
  }
}

template <int L, typename T>
__device__ __forceinline__ T lane_pair_t(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, lane_pair<L>(__builtin_bit_cast(int, v)));
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)lane_pair<L>((int)(unsigned)b);
    const unsigned hi = (unsigned)lane_pair<L>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

template <int SEG, typename T, int L = 0>
__device__ __forceinline__ T seg_max(T v) {
  if constexpr ((2 << L) <= SEG) {
    const T o = lane_pair_t<L>(v);
    return seg_max<SEG, T, L + 1>(o > v ? o : v);
  } else {
    return v;
  }
}

// Arg-max over the segment of (v, smallest key on ties); bl carries the
// winning lane.  The order is total, so the winner does not depend on the
// pairing.
template <int SEG, typename T, int L = 0>
__device__ __forceinline__ void seg_argmax(T& v, int& key, int& bl) {
  if constexpr ((2 << L) <= SEG) {
    const T ov = lane_pair_t<L>(v);
    const int ok = lane_pair<L>(key);
    const int ol = lane_pair<L>(bl);
    const bool take = (ov > v) || (ov == v && ok < key);
    v = take ? ov : v;
    key = take ? ok : key;
    bl = take ? ol : bl;
    seg_argmax<SEG, T, L + 1>(v, key, bl);
  }
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// val from lane src of this lane's segment (src the same for every lane of
// the segment).  A whole-wave segment reads it with v_readlane, a short VALU
// latency on the serial chains of the triangular solves (such kernels run at
// one wave per SIMD); smaller segments, whose kernels keep more waves per
// SIMD to cover the latency, use one crossbar shuffle.
template <int SEG, typename T>
__device__ __forceinline__ T seg_bcast(T val, int seg_base, int src) {
  if constexpr (SEG == 64) {
    return readlane_t(val, __builtin_amdgcn_readfirstlane(src) & 63);
  } else {
    return __shfl(val, seg_base + src, 64);
  }
}

template <int SEG, typename T>
__device__ __forceinline__ T seg_sum(T v) {
#pragma unroll
  for (int off = SEG / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, SEG);
  return v;
}

// NC: columns each lane holds (a multiple of CH, at most SEG): blocks of n
// <= NC rows use NC columns, and the lanes of the segment past NC hold no
// row and never pivot.
template <int SEG, typename T, int NC = SEG>
struct SpcLU {
  static constexpr int CH = SEG < 8 ? SEG : 8;
  static constexpr int NCH = NC / CH;
  static_assert(NC % CH == 0 && NC <= SEG, "row width");

  __device__ static __forceinline__ void rotl(T (&row)[NC]) {
    if (NCH == 1) return;
    T tmp[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) tmp[c] = row[c];
#pragma unroll
    for (int j = 0; j < NC - CH; ++j) row[j] = row[j + CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) row[NC - CH + c] = tmp[c];
  }

  __device__ static __forceinline__ void rotr(T (&row)[NC]) {
    if (NCH == 1) return;
    T tmp[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) tmp[c] = row[NC - CH + c];
#pragma unroll
    for (int j = NC - 1; j >= CH; --j) row[j] = row[j - CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) row[c] = tmp[c];
  }

  // Factor the lane-held rows in place (n <= SEG real rows, the rest are
  // identity).  prow: SEG values of LDS for this segment; wl: SEG ints of LDS
  // for this segment, receives the lane holding each position.  On return
  // row[] holds this lane's row of L\U in column order, pos its position in
  // the permuted matrix, piv the LAPACK pivot of step k == r.  Returns info
  // (1-based first exactly-zero pivot, 0 if none).
  __device__ static __forceinline__ int factor(T (&row)[NC], int r, int n, int& pos, int& piv, T* prow,
                               int* wl) {
    pos = r;
    piv = r;
    bool done = r >= NC;
    int info = 0;
    const int nch = (n + CH - 1) / CH;
    for (int c = 0; c < NCH; ++c) {
      if (c < nch) {
        const int lim = NC - c * CH;    // rotated columns >= lim hold L of earlier chunks
#pragma unroll
        for (int kk = 0; kk < CH; ++kk) {
          const int k = c * CH + kk;
          // NaN ranks above every number so that all lanes of the segment
          // agree on one winner (the comparison below is then a total order)
          T v = done ? T(-1) : sabs(row[kk]);
          if (!(v == v)) v = T(__builtin_inf());
          int key = done ? 0x7fffffff : pos;
          int bl = r;
          seg_argmax<SEG>(v, key, bl);
          if (r == k) piv = key;
          // Columns at or past lim hold multipliers of earlier chunks: the
          // pivot row is published, and the other rows updated, only over
          // the groups of CH columns before lim (a uniform branch per group).
          if (r == bl) {
            prow[kk] = row[kk];
#pragma unroll
            for (int j = kk + 1; j < CH; ++j) prow[j] = row[j];
#pragma unroll
            for (int g = 1; g < NCH; ++g)
              if (g * CH < lim)
#pragma unroll
                for (int j = g * CH; j < (g + 1) * CH; ++j) prow[j] = row[j];
            wl[k] = bl;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const T d = prow[kk];
          if (pos == k) pos = key;
          if (r == bl) {
            pos = k;
            done = true;
          }
          if (d == T(0)) {
            if (!info) info = k + 1;
          } else if (!done) {
            const T l = row[kk] / d;
            row[kk] = l;
#pragma unroll
            for (int j = kk + 1; j < CH; ++j) row[j] = fma(-l, prow[j], row[j]);
#pragma unroll
            for (int g = 1; g < NCH; ++g)
              if (g * CH < lim)
#pragma unroll
                for (int j = g * CH; j < (g + 1) * CH; ++j) row[j] = fma(-l, prow[j], row[j]);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      rotl(row);
    }
    return info;
  }

  // Solve with factors from factor() (pos, wl) or, with wl == nullptr, with
  // factors already in position order (lane r holds position r).  `val` is
  // this lane's right-hand-side entry, already permuted in the second case.
  // Returns component r of the solution.  row[] is left unchanged.
  __device__ static __forceinline__ T solve(T (&row)[NC], int r, int seg_base, int n, int pos, const int* wl,
                            T val) {
    const int nch = (n + CH - 1) / CH;
    for (int c = 0; c < NCH; ++c) {
      if (c < nch) {
#pragma unroll
        for (int kk = 0; kk < CH; ++kk) {
          const int k = c * CH + kk;
          const int src = wl ? wl[k] : k;
          const T yk = seg_bcast<SEG>(val, seg_base, src);
          if (pos > k) val = fma(-row[kk], yk, val);
        }
      }
      rotl(row);
    }
    T x = T(0);
    for (int c = NCH - 1; c >= 0; --c) {
      rotr(row);
      if (c < nch) {
#pragma unroll
        for (int kk = CH - 1; kk >= 0; --kk) {
          const int k = c * CH + kk;
          if (pos == k) val = val / row[kk];
          const int src = wl ? wl[k] : k;
          const T xk = seg_bcast<SEG>(val, seg_base, src);
          if (pos < k) val = fma(-row[kk], xk, val);
          if (r == k) x = xk;
        }
      }
    }
    return x;
  }

  // solve() for factors in position order (lane r holds position r, val
  // already permuted), for the FP32 solves that iterative refinement
  // corrects: the substitutions are unrolled over all NC columns (static
  // register indices without the rotations, a fixed source lane at every
  // step, one uniform branch per chunk of CH columns skipping the chunks past
  // n), each step is branch-free (selects), and the back substitution
  // multiplies by the reciprocal of the pivot, dinv = 1 / U_rr of this lane
  // (pivot_reciprocal), in place of the division.
  __device__ static __forceinline__ T solve_ordered(T (&row)[NC], int r, int seg_base, int n,
                                                    T dinv, T val) {
    const int nch = (n + CH - 1) / CH;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      if (c < nch) {
#pragma unroll
        for (int kk = 0; kk < CH; ++kk) {
          const int k = c * CH + kk;
          const T yk = seg_bcast<SEG>(val, seg_base, k);
          const T u = fma(-row[k], yk, val);
          val = r > k ? u : val;
        }
      }
    }
    T x = T(0);
#pragma unroll
    for (int c = NCH - 1; c >= 0; --c) {
      if (c < nch) {
#pragma unroll
        for (int kk = CH - 1; kk >= 0; --kk) {
          const int k = c * CH + kk;
          const T xk = seg_bcast<SEG>(val, seg_base, k) * seg_bcast<SEG>(dinv, seg_base, k);
          const T u = fma(-row[k], xk, val);
          val = r < k ? u : val;
          x = r == k ? xk : x;
        }
      }
    }
    return x;
  }

  // 1 / U_rr of this lane's row in position order (1 on rows past n and on
  // lanes without a row; an exactly zero pivot gives an infinity, as the
  // division would).
  __device__ static __forceinline__ T pivot_reciprocal(const T (&row)[NC], int r) {
    T d = T(1);
#pragma unroll
    for (int j = 0; j < NC; ++j) d = r == j ? row[j] : d;
    return T(1) / d;
  }

  // Lane (within the segment) that holds position r after factor(): the
  // pivot lane of step r for the factored chunks, r itself past them
  // (identity rows of padding lanes, never exchanged).
  __device__ static __forceinline__ int position_source(int r, int n, const int* wl) {
    const int nk = (n + CH - 1) / CH * CH;
    return r < nk ? wl[r] : r;
  }

  // Move the rows of factor() into position order (lane r then holds the row
  // of position r, for solve_ordered with the right-hand side read from lane
  // src first), so that every substitution step reads a fixed lane.  src:
  // position_source(r, ...).
  __device__ static __forceinline__ void to_position_order(T (&row)[NC], int seg_base, int src) {
#pragma unroll
    for (int j = 0; j < NC; ++j) row[j] = __shfl(row[j], seg_base + src, 64);
  }

  // Solve with factors stored in LAPACK layout (lane r holds the row at
  // position r) and LAPACK pivots piv[0..n-1] in global memory.
  __device__ static __forceinline__ T solve_stored(T (&row)[NC], int r, int seg_base, const int* piv, int n,
                                   T val) {
    for (int k = 0; k < n; ++k) {
      const int p = piv[k];
      const T vk = __shfl(val, seg_base + k, 64);
      const T vp = __shfl(val, seg_base + p, 64);
      if (r == k)
        val = vp;
      else if (r == p)
        val = vk;
    }
    return solve(row, r, seg_base, n, r, nullptr, val);
  }
};

// Segment-per-cell explicit inverse by Gauss-Jordan elimination, in place
// and one row per lane as in SpcLU.  Step k takes the pivot as factor() does
// (first maximal |a| among the rows not yet pivoted), divides the pivot row
// by it and subtracts multiples of it from every other row, so that column k
// becomes a unit vector; the freed column then holds the new column of the
// inverse (the right half of Gauss-Jordan on [A | I], kept in the left
// half's place).  The divisions of the pivot row are spread over the lanes,
// one entry each.
template <int SEG, int NC = SEG>
struct SpcGJ {
  static constexpr int CH = SEG < 8 ? SEG : 8;
  static constexpr int NCH = NC / CH;
  static_assert(NC % CH == 0 && NC <= SEG, "row width");

  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // Invert the lane-held rows in place (n <= NC real rows, identity rows
  // past n).  prow: SEG doubles of LDS for this segment, wl: SEG ints of LDS
  // (receives the lane holding each position).  On return lane r holds, in
  // position order of its columns, the row of the inverse of the
  // row-permuted block PA for unknown pos: x[pos] = sum_j row[j] (P b)_j with
  // (P b)_j the right-hand side of the row at position j.  Returns info
  // (1-based first exactly-zero pivot, 0 if none).
  __device__ static __forceinline__ int invert(double (&row)[NC], int r, int n, int& pos,
                                               double* prow, int* wl) {
    pos = r;
    bool done = r >= NC;
    const bool held = r < NC;
    int info = 0;
    const int nch = (n + CH - 1) / CH;
    for (int c = 0; c < NCH; ++c) {
      if (c < nch) {
#pragma unroll
        for (int kk = 0; kk < CH; ++kk) {
          const int k = c * CH + kk;
          double v = done ? -1.0 : sabs(row[kk]);
          if (!(v == v)) v = __builtin_inf();
          int key = done ? 0x7fffffff : pos;
          int bl = r;
          seg_argmax<SEG>(v, key, bl);
          if (r == bl) {
#pragma unroll
            for (int j = 0; j < NC; ++j) prow[j] = row[j];
            wl[k] = bl;
          }
          sync();
          const double d = prow[kk];
          // lane t divides entry t of the pivot row; the entry of column k
          // becomes the new inverse column's 1 / d
          double e = 0.0;
          if (held) e = (r == kk ? 1.0 : prow[r]) / d;
          sync();
          if (held) prow[r] = e;
          sync();
          if (pos == k) pos = key;
          if (r == bl) {
            pos = k;
            done = true;
          }
          if (d == 0.0) {
            if (!info) info = k + 1;
          } else if (held) {
            // the pivot row is read 16 columns at a time (the empty asm keeps
            // the next group's LDS reads after this group's update, so they
            // do not all wait in registers at once)
            const double f = row[kk];
            const bool piv_row = r == bl;
#pragma unroll
            for (int j0 = 0; j0 < NC; j0 += 16) {
#pragma unroll
              for (int j = j0; j < j0 + 16 && j < NC; ++j) {
                const double pj = prow[j];
                row[j] = piv_row ? pj : (j == kk ? -f * pj : fma(-f, pj, row[j]));
              }
              asm volatile("" ::: "memory");
            }
          }
          sync();
        }
      }
      if constexpr (NCH > 1) {   // rotate left by CH (see SpcLU)
        double tmp[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) tmp[q] = row[q];
#pragma unroll
        for (int j = 0; j < NC - CH; ++j) row[j] = row[j + CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) row[NC - CH + q] = tmp[q];
      }
    }
    return info;
  }

  // x_r = sum_m X[r][m] b_m with row r of the inverse in natural column order
  // in this lane (b_m from lane m of the segment: v_readlane for a
  // whole-wave segment, an LDS broadcast otherwise).  prow: SEG doubles of
  // LDS for the segment.  Lanes past NC return 0.
  __device__ static __forceinline__ double apply_natural(const double (&X)[NC], int r, double b,
                                                         int seg_base, double* prow) {
    double s = 0.0;
    if constexpr (SEG == 64) {
#pragma unroll
      for (int m = 0; m < NC; ++m) s = fma(X[m], readlane_t(b, m), s);
    } else {
      __builtin_amdgcn_wave_barrier();
      prow[r] = b;
      sync();
#pragma unroll
      for (int m = 0; m < NC; ++m) s = fma(X[m], prow[m], s);
      sync();
    }
    (void)seg_base;
    return r < NC ? s : 0.0;
  }

  // x for this lane's unknown r from the rows invert() left (row, pos) and
  // this lane's right-hand-side entry b: the right-hand sides are placed by
  // position, each lane forms its inverse row's sum in position order, and
  // the sums return to the lanes of their unknowns.  prow: SEG doubles of
  // LDS for the segment.  Lanes past NC return 0.
  __device__ static __forceinline__ double apply(const double (&row)[NC], int r, int pos, double b,
                                                 double* prow) {
    const bool held = r < NC;
    __builtin_amdgcn_wave_barrier();
    if (held) prow[pos] = b;
    sync();
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) s = fma(row[j], prow[j], s);
    sync();
    if (held) prow[pos] = s;
    sync();
    const double x = held ? prow[r] : 0.0;
    sync();
    return x;
  }
};

}  // namespace bdfgpu
