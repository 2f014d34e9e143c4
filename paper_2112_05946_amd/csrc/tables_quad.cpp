// Operand tables of the matrix-core stage kernel for quadrilaterals: the chaos
// basis at the random nodes (Sec. 2.1, Eq. polynomial chaos) and the
// quadrature-weighted basis (Eq. discrete expectation value) arranged as the
// per-lane A operands of the 16 x 16 matrix instructions, so that a lane loads
// its operand with one coalesced access.
//
// Lane l of a wave holds, for the FP64 instruction (16 x 16 x 4, A[i][k] in
// lane i + 16 k): row i = l % 16, column k = l / 16; for the bfloat16
// instruction (16 x 16 x 16, A[i][k] in lane i + 16 (k / 4), item k % 4): row
// i = l % 16, columns 4 (l / 16) .. 4 (l / 16) + 3.
//
// Random nodes come in blocks of 16; in node block nb, lane group g and
// register r of an instruction's result hold node 16 nb + g + 4 r, so that
// the nodes past N_q (padding up to a multiple of 16) fill whole registers.
// A padded node repeats node 0 in the expansion tables (its values stay a
// physical state) and carries weight 0 in the projection tables.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "internal.hpp"

namespace frsg {
namespace {

uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
// x = hi + lo to about 16 significant bits, both parts bfloat16
void split_bf16(double x, uint16_t& hi, uint16_t& lo) {
  const float f = (float)x;
  hi = bf16_rne(f);
  lo = bf16_rne(f - bf16_value(hi));
}
double pack4(const uint16_t* v) {
  uint64_t u = (uint64_t)v[0] | ((uint64_t)v[1] << 16) | ((uint64_t)v[2] << 32) | ((uint64_t)v[3] << 48);
  double d;
  std::memcpy(&d, &u, 8);
  return d;
}

}  // namespace

void build_quad_fragments(HostTables& T) {
  const int M = T.M, Nq = T.Nq;
  const QuadFragLayout L = quad_frag_layout(Nq);
  std::vector<double>& F = T.qfrag;
  F.assign(L.total, 0.0);
  auto phi = [&](int k, int q) { return (k < M) ? T.Phi[k * Nq + (q < Nq ? q : 0)] : 0.0; };
  auto pw = [&](int k, int q) { return (k < M && q < Nq) ? T.PW[k * Nq + q] : 0.0; };
  for (int nb = 0; nb < L.nb; ++nb) {
    for (int l = 0; l < 64; ++l) {
      const int i = l % 16, c = l / 16;
      for (int t = 0; t < 4; ++t) {
        // FP64 instruction, result row i = node 16 nb + i (lane group i % 4, register i / 4)
        F[L.aexp_f + (nb * 4 + t) * 64 + l] = phi(4 * t + c, 16 * nb + i);  // mode 4 t + k
        F[L.aexp_b + (nb * 4 + t) * 64 + l] = phi(4 * c + t, 16 * nb + i);  // mode 4 k + t
        // projection: result row i = mode i, column k = node 16 nb + k + 4 r
        F[L.aprj + (nb * 4 + t) * 64 + l] = pw(i, 16 * nb + c + 4 * t);
      }
      // bfloat16 instruction, result row i in lane group i / 4, register i % 4:
      // row i = node 16 nb + i / 4 + 4 (i % 4)
      uint16_t eh[4], el[4], ph[4], pl[4];
      for (int it = 0; it < 4; ++it) {
        const int kk = 4 * c + it;  // column of the A operand
        split_bf16(phi(kk, 16 * nb + i / 4 + 4 * (i % 4)), eh[it], el[it]);
        split_bf16(pw(i, 16 * nb + kk / 4 + 4 * (kk % 4)), ph[it], pl[it]);
      }
      F[L.bexp + (nb * 2 + 0) * 64 + l] = pack4(eh);
      F[L.bexp + (nb * 2 + 1) * 64 + l] = pack4(el);
      F[L.bprj + (nb * 2 + 0) * 64 + l] = pack4(ph);
      F[L.bprj + (nb * 2 + 1) * 64 + l] = pack4(pl);
    }
    for (int r = 0; r < 4; ++r)
      for (int g = 0; g < 4; ++g) {
        const int q = 16 * nb + g + 4 * r;
        F[L.wslot + nb * 16 + r * 4 + g] = (q < Nq) ? T.wq[q] : 0.0;
      }
  }
}

}  // namespace frsg
