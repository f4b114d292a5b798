// row_vi.hip -- the value-iteration sweep (Eq. (18), Alg. 3 step 2) in the
// row form of the tile sweep.
//
// The tiles are those of the tile form with T = 3 low digits: the R^3
// occupancies (R = C + 1) that share the high digits n_3..n_{K-1}, staged in
// LDS by one workgroup.  Inside a tile each lane owns a chunk of four
// consecutive occupancies of one row along digit 0 (rows are padded to a
// multiple of four slots in LDS; the last chunk of a row holds R mod 4 of
// them).  Against one occupancy per lane this
//  * turns every neighbour along a high digit into one 16-byte load per
//    class (values) or two (arrival terms) at the lane's offset plus a
//    workgroup-uniform offset, instead of four scalar loads;
//  * turns every neighbour along digits 1 and 2 into one 16-byte LDS read
//    per class at a per-lane row base, and along digit 0 into a register of
//    the chunk or one LDS word;
//  * leaves no per-occupancy index arithmetic: the radix is a compile-time
//    constant, the row and chunk of a lane fix its digits, and a placement
//    past the last slot of a row lands on -inf padding.
// Per state the arithmetic and its order are those of the other forms, so the
// iterates are bit-identical to theirs.
#include "kernels.hpp"
#include "row.hpp"

namespace mdpvi {

#ifndef MDPVI_ROW_CLASS_UNROLL
#define MDPVI_ROW_CLASS_UNROLL 0
#endif

template <int K, int J, int R>
__global__ __launch_bounds__((RowGeo<R, 4>::BLOCK), MDPVI_ROW_WAVES) void vi_row_kernel(Model M, TileShape S, const float* __restrict__ Vin,
                                                                  float* __restrict__ Vout,
                                                                  const double* __restrict__ Ain,
                                                                  double* __restrict__ Aout, Ctl* ctl, double* res,
                                                                  long long j, double tol) {
  using G = RowGeo<R, 4>;
  constexpr int T = 3;
  constexpr int NH = K - T;
  if (sweep_stopped<ResKind::kMax>(ctl, res, j, tol)) return;
  // arrival terms [ROWS + 1][RPA] (the last row all -inf), values [J][ROWS][RP]
  __shared__ __align__(16) double Al[(G::ROWS + 1) * G::RPA];
  __shared__ __align__(16) float Vl[J * G::ROWS * G::RP];
  const uint32_t nocc = static_cast<uint32_t>(M.n_occ);
  const uint32_t ns = static_cast<uint32_t>(M.n_states);
  const uint32_t cls = nocc * 4u;
  const BufView vin = make_view(Vin, ns * 4u);
  const BufView vout = make_view(Vout, ns * 4u);
  const BufView ain = make_view(Ain, (nocc + kSentinel) * 8u);
  const BufView aout = make_view(Aout, nocc * 8u);
  // -inf padding that no staging overwrites: the sentinel row and the slots
  // past the last chunk of every row
  for (int t = threadIdx.x; t < G::RPA; t += G::BLOCK) Al[G::ROWS * G::RPA + t] = -INFINITY;
  if constexpr (G::RPA > G::RP) {
    for (int t = threadIdx.x; t < G::ROWS * (G::RPA - G::RP); t += G::BLOCK)
      Al[(t / (G::RPA - G::RP)) * G::RPA + G::RP + t % (G::RPA - G::RP)] = -INFINITY;
  }
  const int lane = static_cast<int>(threadIdx.x);
  const bool act = lane < G::LANES;
  const int r = act ? lane / G::NC : 0;       // row of the tile: digits 1 and 2
  const int c = act ? lane % G::NC : 0;       // chunk of the row
  const int n1 = r % R, n2 = r / R;
  const int c4 = 4 * c;                       // digit 0 of the chunk's first occupancy
  const bool tail = c == G::NC - 1;           // the row's last chunk (TAIL occupancies)
  const uint32_t loff = static_cast<uint32_t>(r * R + c4);   // element offset in the tile
  const uint32_t lo4 = loff * 4u, lo8 = loff * 8u;
  // per-lane weights that do not depend on the tile
  const double mu1 = M.mu_L * n1, mu2 = M.mu_L * n2;
  // LDS rows of the digit-1 and digit-2 neighbours
  const int rd1 = n1 > 0 ? r - 1 : r, rr1 = r - n1;
  const int rd2 = n2 > 0 ? r - R : r, rr2 = r - n2 * R;
  double dmax = 0.0;
  bool bad = false;
  const TileWalk tw = tile_walk(S);
  for (uint32_t tp = tw.first; tp < tw.end; tp += tw.step) {
    const uint32_t tb = tile_at(S, tp);
    TileHigh<K, J, T> H;
    tile_high_setup<K, J, T>(M, tb, H);
    const bool last_tile = tb + 1 == S.n;
    // ---- stage the tile: values of every class and the arrival terms
    if (act) {
      float v[J][4];
#pragma unroll
      for (int e = 0; e < J; ++e) {
        // the array's last chunk has no fourth element to read
        if (e == J - 1 && last_tile && r == G::ROWS - 1 && tail)
          ld3f(vin, lo4, H.o0 * 4u + e * cls, v[e]);
        else
          ld4f(vin, lo4, H.o0 * 4u + e * cls, v[e]);
      }
      double a[4];
      ld4d(ain, lo8, H.o0 * 8u, a);
      if (tail) {
#pragma unroll
        for (int p = G::TAIL; p < 4; ++p) a[p] = -INFINITY;
      }
#pragma unroll
      for (int e = 0; e < J; ++e)
        *reinterpret_cast<float4*>(&Vl[(e * G::ROWS + r) * G::RP + c4]) = make_float4(v[e][0], v[e][1], v[e][2], v[e][3]);
      *reinterpret_cast<double2*>(&Al[r * G::RPA + c4]) = make_double2(a[0], a[1]);
      *reinterpret_cast<double2*>(&Al[r * G::RPA + c4 + 2]) = make_double2(a[2], a[3]);
    }
    __syncthreads();
    if (act) {
      const int load0 = H.load_high + n1 + n2 + c4;   // units in use at the chunk's first occupancy
      double muh[NH > 0 ? NH : 1];
#pragma unroll
      for (int h = 0; h < NH; ++h) muh[h] = M.mu_L * H.nh[h];
      double anew[4] = {0.0, 0.0, 0.0, 0.0};
      const bool full = !tail || G::TAIL == 4;
#if MDPVI_ROW_CLASS_UNROLL
#pragma unroll
#else
#pragma unroll 1
#endif
      for (int e = 0; e < J; ++e) {
        const int s = M.size[e];
        // neighbours along the high digits (global memory), in flight while
        // the in-tile part of the backup runs
        float gd[NH > 0 ? NH : 1][4], gr[NH > 0 ? NH : 1][4];
        double ga[NH > 0 ? NH : 1][4];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const uint32_t st = static_cast<uint32_t>(M.stride[T + h]);
          const uint32_t ha8 = H.nh[h] + s <= M.C ? (H.o0 + static_cast<uint32_t>(s) * st) * 8u : nocc * 8u;
          ld4f(vin, lo4, H.hd4[h] + e * cls, gd[h]);
          ld4f(vin, lo4, H.hr4[h] + e * cls, gr[h]);
          ld4d(ain, lo8, ha8, ga[h]);
        }
        const float* Ve = &Vl[e * G::ROWS * G::RP];
        const float4 x_s = *reinterpret_cast<const float4*>(&Ve[r * G::RP + c4]);
        const float vs[4] = {x_s.x, x_s.y, x_s.z, x_s.w};
        // digit 0: release from the previous slot (the state itself at n_0 = 0,
        // weight 0), reset to the row's first slot
        const float vprev = c4 > 0 ? Ve[r * G::RP + c4 - 1] : vs[0];
        const double vrow0 = static_cast<double>(Ve[r * G::RP]);
        // in-tile part of the sums: digits 0, 1, 2 in order
        double D[4], rs[4], ab[4];
        {
          const double* a0 = &Al[r * G::RPA + c4 + s];   // slot n_0 + s; -inf padding past the row
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const double idle = M.mu_L * static_cast<double>(M.KC - (load0 + p));
            D[p] = idle * static_cast<double>(vs[p]);
            D[p] = fma(M.mu_L * (c4 + p), static_cast<double>(p > 0 ? vs[p - 1] : vprev), D[p]);
            rs[p] = 0.0 + vrow0;
            ab[p] = a0[p];
          }
        }
        {
          const float4 d1 = *reinterpret_cast<const float4*>(&Ve[rd1 * G::RP + c4]);
          const float4 q1 = *reinterpret_cast<const float4*>(&Ve[rr1 * G::RP + c4]);
          const int ra1 = n1 + s <= M.C ? r + s : G::ROWS;   // the sentinel row without room
          const double2 x = *reinterpret_cast<const double2*>(&Al[ra1 * G::RPA + c4]);
          const double2 y = *reinterpret_cast<const double2*>(&Al[ra1 * G::RPA + c4 + 2]);
          const float vd[4] = {d1.x, d1.y, d1.z, d1.w}, vr[4] = {q1.x, q1.y, q1.z, q1.w};
          const double aa[4] = {x.x, x.y, y.x, y.y};
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            D[p] = fma(mu1, static_cast<double>(vd[p]), D[p]);
            rs[p] += static_cast<double>(vr[p]);
            ab[p] = max_f64(ab[p], aa[p]);
          }
        }
        {
          const float4 d2 = *reinterpret_cast<const float4*>(&Ve[rd2 * G::RP + c4]);
          const float4 q2 = *reinterpret_cast<const float4*>(&Ve[rr2 * G::RP + c4]);
          const int ra2 = n2 + s <= M.C ? r + s * R : G::ROWS;
          const double2 x = *reinterpret_cast<const double2*>(&Al[ra2 * G::RPA + c4]);
          const double2 y = *reinterpret_cast<const double2*>(&Al[ra2 * G::RPA + c4 + 2]);
          const float vd[4] = {d2.x, d2.y, d2.z, d2.w}, vr[4] = {q2.x, q2.y, q2.z, q2.w};
          const double aa[4] = {x.x, x.y, y.x, y.y};
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            D[p] = fma(mu2, static_cast<double>(vd[p]), D[p]);
            rs[p] += static_cast<double>(vr[p]);
            ab[p] = max_f64(ab[p], aa[p]);
          }
        }
        // high digits in order
#pragma unroll
        for (int h = 0; h < NH; ++h) {
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            D[p] = fma(muh[h], static_cast<double>(gd[h][p]), D[p]);
            rs[p] += static_cast<double>(gr[h][p]);
            ab[p] = max_f64(ab[p], ga[h][p]);
          }
        }
        double a_rej[4];   // the paid cloud: the arrival term at n itself
        {
          const double2 x = *reinterpret_cast<const double2*>(&Al[r * G::RPA + c4]);
          const double2 y = *reinterpret_cast<const double2*>(&Al[r * G::RPA + c4 + 2]);
          a_rej[0] = x.x; a_rej[1] = x.y; a_rej[2] = y.x; a_rej[3] = y.y;
        }
        float vn[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const double Dp = fma(M.nu_L, rs[p], D[p]);
          const double fu = static_cast<double>(M.KC - (load0 + p));
          const double best = max_f64(fma(M.gamma, a_rej[p], fma(-M.hold, fu, M.r_reject[e])),
                                      fma(M.gamma, ab[p], fma(-M.hold, fu, M.r_place[e])));
          vn[p] = static_cast<float>(fma(M.gamma, Dp, best));
          anew[p] = fma(M.p[e], static_cast<double>(vn[p]), anew[p]);
          if (!tail || p < G::TAIL) {
            const double dd = fabs(static_cast<double>(vn[p]) - static_cast<double>(vs[p]));
            dmax = dd > dmax ? dd : dmax;
            bad = bad || (dd != dd);
          }
        }
        // store the class's chunk (the row's last chunk holds TAIL occupancies)
        const uint32_t uo = H.o0 * 4u + e * cls;
        if (full) {
          const U32x4 x = {__float_as_uint(vn[0]), __float_as_uint(vn[1]), __float_as_uint(vn[2]),
                           __float_as_uint(vn[3])};
          __builtin_amdgcn_raw_buffer_store_b128(x, vout.r, lo4, uo, 0);
        } else if constexpr (G::TAIL == 3) {
          const U32x3 x = {__float_as_uint(vn[0]), __float_as_uint(vn[1]), __float_as_uint(vn[2])};
          __builtin_amdgcn_raw_buffer_store_b96(x, vout.r, lo4, uo, 0);
        } else if constexpr (G::TAIL == 2) {
          const U32x2v x = {__float_as_uint(vn[0]), __float_as_uint(vn[1])};
          __builtin_amdgcn_raw_buffer_store_b64(x, vout.r, lo4, uo, 0);
        } else {
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vn[0]), vout.r, lo4, uo, 0);
        }
      }
      {
        const uint32_t uo = H.o0 * 8u;
        const U32x4 x = {lo32(anew[0]), hi32(anew[0]), lo32(anew[1]), hi32(anew[1])};
        const U32x4 y = {lo32(anew[2]), hi32(anew[2]), lo32(anew[3]), hi32(anew[3])};
        if (full) {
          __builtin_amdgcn_raw_buffer_store_b128(x, aout.r, lo8, uo, 0);
          __builtin_amdgcn_raw_buffer_store_b128(y, aout.r, lo8 + 16u, uo, 0);
        } else if constexpr (G::TAIL == 3) {
          __builtin_amdgcn_raw_buffer_store_b128(x, aout.r, lo8, uo, 0);
          const U32x2v z = {lo32(anew[2]), hi32(anew[2])};
          __builtin_amdgcn_raw_buffer_store_b64(z, aout.r, lo8 + 16u, uo, 0);
        } else if constexpr (G::TAIL == 2) {
          __builtin_amdgcn_raw_buffer_store_b128(x, aout.r, lo8, uo, 0);
        } else {
          const U32x2v z = {lo32(anew[0]), hi32(anew[0])};
          __builtin_amdgcn_raw_buffer_store_b64(z, aout.r, lo8, uo, 0);
        }
      }
    }
    __syncthreads();   // the next tile overwrites the LDS image
  }
  block_max_to<G::BLOCK>(bad ? NAN : dmax, ctl, res, j, tol);
}

bool vi_row_shape(const Model& M, TileShape* S) {
  if (M.K < 5 || M.K > 7 || M.R != 11 || M.J < 1 || M.J > 3 || M.n_sizes != M.J) return false;
  for (int e = 0; e < M.J; ++e)
    if (M.size[e] > RowGeo<11, 4>::MAXS) return false;
  if (!tile_shape(M, 4u * M.J + 8u, kTileLds, S) || S->T != 3) return false;
  return true;
}

hipError_t launch_vi_row(const Model& M, const TileShape& S, const float* Vin, float* Vout, const double* Ain,
                         double* Aout, Ctl* ctl, double* res, long long j, double tol, hipStream_t s) {
  return row_dispatch(M.K, M.J, M.R, [&](auto kc, auto jc, auto rc) {
    constexpr int Kc = decltype(kc)::value, Jc = decltype(jc)::value, Rc = decltype(rc)::value;
    hipLaunchKernelGGL((vi_row_kernel<Kc, Jc, Rc>), dim3(S.grid), dim3((RowGeo<Rc, 4>::BLOCK)), 0, s, M, S, Vin, Vout,
                       Ain, Aout, ctl, res, j, tol);
    return hipGetLastError();
  });
}

}  // namespace mdpvi
