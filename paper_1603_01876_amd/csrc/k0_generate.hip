// k0_generate.hip -- K0, the Kronecker edge generator (Sec. IV.A).
//
// Edge e is a pure function of (e, parameters): level l of its raw labels
// is a 2x2 quadrant drawn with probabilities a, b, c, d from Philox4x32-10
// at counter (e mod 2^32, e div 2^32, l div 2, 0), one block serving two
// levels; the raw labels are then relabelled by a keyed bijection on S bits.
// No communication, no workspace: one thread per edge in a grid-stride loop,
// two coalesced int64 stores per edge.  The kernel is ALU-bound (Philox),
// which is why labels are built in 32-bit registers.
#include "pp_common.hpp"

#include <cmath>

namespace pp {

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): Weyl increment, then a
// xor-shift-multiply finaliser.  Host-side only; feeds the relabelling keys.
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// Probability -> 32-bit integer threshold: round(p * 2^32), ties up,
// clamped to [0, 2^32 - 1].
uint32_t threshold(double p) {
  const double x = std::ldexp(p, 32);
  if (!(x > 0.0)) return 0u;
  const double y = std::floor(x + 0.5);
  return y >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(y);
}

struct GenArgs {
  int64_t m;
  int32_t scale;
  uint32_t mask;       // 2^S - 1
  int32_t half;        // max(1, S/2): xor-shift of the relabelling rounds
  uint32_t t_u;        // P(u-bit = 1) = c + d
  uint32_t t_v0;       // P(v-bit = 1 | u-bit = 0) = b / (a + b)
  uint32_t t_v1;       // P(v-bit = 1 | u-bit = 1) = d / (c + d)
  uint32_t key0, key1; // Philox key = seed
  uint32_t mul[4];     // odd multipliers of the relabelling rounds
  uint32_t add[4];
};

__device__ __forceinline__ uint32_t relabel(uint32_t x, const GenArgs &g) {
  // (x*m + a) mod 2^S computed mod 2^32 then masked: 2^S divides 2^32.
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    x = (x * g.mul[r] + g.add[r]) & g.mask;
    x ^= x >> g.half;
  }
  return x;
}

__global__ __launch_bounds__(256) void k_generate(GenArgs g, int64_t *__restrict__ u,
                                                  int64_t *__restrict__ v) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < g.m; e += stride) {
    uint32_t uu = 0, vv = 0;
    const uint32_t elo = uint32_t(e), ehi = uint32_t(uint64_t(e) >> 32);
    for (int32_t j = 0; 2 * j < g.scale; ++j) {
      const U4 w = philox10(U4{elo, ehi, uint32_t(j), 0u}, g.key0, g.key1);
      // level 2j: draws (x, y) = words 0, 1
      {
        const uint32_t ub = w.x < g.t_u;
        const uint32_t vb = w.y < (ub ? g.t_v1 : g.t_v0);
        uu |= ub << (2 * j);
        vv |= vb << (2 * j);
      }
      // level 2j+1: draws (x, y) = words 2, 3
      if (2 * j + 1 < g.scale) {
        const uint32_t ub = w.z < g.t_u;
        const uint32_t vb = w.w < (ub ? g.t_v1 : g.t_v0);
        uu |= ub << (2 * j + 1);
        vv |= vb << (2 * j + 1);
      }
    }
    u[e] = int64_t(relabel(uu, g));
    v[e] = int64_t(relabel(vv, g));
  }
}

}  // namespace

pp_status launch_generate(const pp_kron_params &p, int64_t *u, int64_t *v, hipStream_t s) {
  GenArgs g{};
  g.m = int64_t(p.edge_factor) << p.scale;
  g.scale = p.scale;
  g.mask = p.scale >= 32 ? 0xFFFFFFFFu : ((1u << p.scale) - 1u);
  g.half = p.scale / 2 < 1 ? 1 : p.scale / 2;
  g.t_u = threshold(p.c + p.d);
  g.t_v0 = (p.a + p.b > 0.0) ? threshold(p.b / (p.a + p.b)) : 0u;
  g.t_v1 = (p.c + p.d > 0.0) ? threshold(p.d / (p.c + p.d)) : 0u;
  g.key0 = uint32_t(p.seed);
  g.key1 = uint32_t(p.seed >> 32);
  SplitMix64 sm{p.seed};
  for (int r = 0; r < 4; ++r) {
    g.mul[r] = uint32_t((sm.next() | 1ull) & g.mask);
    g.add[r] = uint32_t(sm.next() & g.mask);
  }
  if (g.m == 0) return PP_OK;
  // 256 CUs x 8 resident workgroups covers the chip; the loop handles the rest.
  hipLaunchKernelGGL(k_generate, dim3(grid_for(g.m, 256, 256 * 16)), dim3(256), 0, s, g, u, v);
  PP_LAUNCHED("k_generate");
  return PP_OK;
}

}  // namespace pp
