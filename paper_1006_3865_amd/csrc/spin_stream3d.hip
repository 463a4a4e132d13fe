// spin_stream3d.hip -- 3D Ising, one whole sweep per launch, streamed over
// planes (the kernel of the L = 512 and 1024 lattices).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_packed.h"
#include "spin_phase.h"

namespace spin {

// 3D Ising, one whole sweep, streaming over planes.  Rows are full x rows,
// L = 512 * G (lane l of a wave owns groups g = l + 64 j, j < G).  A
// workgroup of W waves owns the TY rows [y0, y0+TY) of the planes
// [z0, z0+H) and keeps a ring of 6 plane slices in LDS; a slice holds the
// rows y0-2 .. y0+TY+1 (row r <-> y = y0-2+r), each row with 16 wrap bytes
// on both sides.  Plane k of the strip (z = z0-2+k) lives in slot k % 6.
// Step i (i = 0..H+2), a = z0-1+i:
//   load plane a+2 (registers; stored to LDS at the end of the step);
//   colour 0 on plane a, rows y0-1 .. y0+TY (the tile rows and a one-row
//   ring that colour 1 needs): reads planes a-1..a+1, writes plane a;
//   colour 1 on plane a-2, rows y0 .. y0+TY-1: reads planes a-3..a-1,
//   writes dst;
//   barrier.
// The 2TY+2 row-units of a step are dealt to the waves round-robin.  The
// step loop is unrolled over the ring period (slots compile-time; with z0
// even the plane parities are too).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Rows move between HBM and registers by buffer instructions over the
// lattice's L^3 bytes (at most 2^30; third descriptor word 0x00020000, the
// raw-buffer format of the gfx9 family): the row offset (z L + y) L is a
// scalar operand and the thread's byte offset 8 (lane + 64 j) the vector
// operand, so no per-lane 64-bit address arithmetic remains.
template <int TY, int W, int G>
struct Stream3Ctx {
  static constexpr uint32_t L = 512u * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t RB = L + 32;
  static constexpr uint32_t RP = TY + 4;
  static constexpr uint32_t PB = RP * RB;
  static constexpr int NT = 64 * W;
  static constexpr int RPW = (RP + W - 1) / W;  // plane rows loaded per wave
  __amdgpu_buffer_rsrc_t rsrc, rdst;
  int8_t* ring;
  const uint32_t* bound;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never4, y0, z0, H, lane, wave;

  __device__ __forceinline__ void get_plane(uint32_t z, uint2 (&v)[RPW][G]) const {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const uint32_t rr = wave + W * q;
      if (rr < RP) {
        const uint32_t y = wrap_row(y0 + rr, 2u, L);
        const uint32_t roff = (z * L + y) * L;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rsrc, 8u * (lane + 64 * j), roff, 0);
          v[q][j] = make_uint2(w.x, w.y);
        }
      }
    }
  }
  __device__ __forceinline__ void put_plane(uint32_t slot, const uint2 (&v)[RPW][G]) const {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const uint32_t rr = wave + W * q;
      if (rr < RP) {
        int8_t* row = ring + slot * PB + rr * RB;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const uint32_t g = lane + 64 * j;
          *reinterpret_cast<uint2*>(row + 16 + 8 * g) = v[q][j];
          if (g >= GPR - 2) *reinterpret_cast<uint2*>(row + 8 * (g - (GPR - 2))) = v[q][j];
          if (g < 2) *reinterpret_cast<uint2*>(row + 16 + L + 8 * g) = v[q][j];
        }
      }
    }
  }
};

// One 8-site group of row r (LDS slot PC, z-neighbour slots PM, PP) in colour C.
template <int TY, int W, int G, bool NEVER, uint32_t C, uint32_t PM, uint32_t PC, uint32_t PP>
__device__ __forceinline__ void stream3_group(const Stream3Ctx<TY, W, G>& c, uint32_t r, uint32_t y,
                                              uint32_t z, uint32_t g, uint32_t& o_lo,
                                              uint32_t& o_hi) {
  using X = Stream3Ctx<TY, W, G>;
  constexpr uint32_t L = X::L, GPR = X::GPR, RB = X::RB, PB = X::PB;
  const int8_t* row = c.ring + PC * PB + r * RB + 16;
  const int8_t* zm = c.ring + PM * PB + r * RB + 16;
  const int8_t* zp = c.ring + PP * PB + r * RB + 16;
  const uint2 cc = *reinterpret_cast<const uint2*>(row + 8 * g);
  const uint2 ym = *reinterpret_cast<const uint2*>(row - RB + 8 * g);
  const uint2 yp = *reinterpret_cast<const uint2*>(row + RB + 8 * g);
  const uint2 a2 = *reinterpret_cast<const uint2*>(zm + 8 * g);
  const uint2 b2 = *reinterpret_cast<const uint2*>(zp + 8 * g);
  const uint32_t lw = *reinterpret_cast<const uint32_t*>(row + 8 * g - 4);
  const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8 * g + 8);
  uint32_t rnd[4];
  const uint32_t cbase = (z * L + y) * GPR;  // < 2^27 for L <= 1024
  philox_lane(cbase + g, C ? c.U1 : c.U0, *c.keys, rnd);
  const uint32_t o0[4] = {ym.x, yp.x, a2.x, b2.x}, o1[4] = {ym.y, yp.y, a2.y, b2.y};
  const uint32_t P = (C + y + z) & 1u;
  const uint32_t Sp = unsat_packed<4>(P, cc.x, cc.y, lw, rw, o0, o1);
  uint32_t c0 = cc.x, c1 = cc.y;
  apply_packed<NEVER>(P, c0, c1, Sp, rnd, c.bound, c.never4);
  o_lo = c0;
  o_hi = c1;
}

// Step i of the plane pipeline.  Wave w updates colour-0 rows 1 + w + W q
// (q < N0, rows 1..TY+2 of plane a) and colour-1 rows 2 + w + W q (q < N1,
// rows 2..TY+1 of plane a-2); rows past the end are computed on a valid row
// and not stored, so the compute is straight-line and the units interleave.
template <int TY, int W, int G, bool NEVER, uint32_t S>
__device__ __forceinline__ void stream3_step(const Stream3Ctx<TY, W, G>& c, uint32_t i) {
  using X = Stream3Ctx<TY, W, G>;
  constexpr uint32_t L = X::L, GPR = X::GPR, RB = X::RB, PB = X::PB;
  constexpr int N0 = (TY + 2 + W - 1) / W, N1 = (TY + W - 1) / W;
  const uint32_t H = c.H;
  if (i >= H + 3) return;
  uint2 nxt[X::RPW][G];
  const bool do_load = (i <= H);
  if (do_load) c.get_plane(wrap_row(c.z0 + i + 3, 2u, L), nxt);
  const bool col0 = (i <= H + 1), col1 = (i >= 3);
  const uint32_t za = wrap_row(c.z0 + i + 1, 2u, L);  // plane a = z0 - 1 + i
  const uint32_t zb = c.z0 + i - 3u;                   // plane a - 2
  uint32_t r0[N0], r1[N1], y0v[N0], y1v[N1];
#pragma unroll
  for (int q = 0; q < N0; ++q) {
    const uint32_t rr = 1u + c.wave + W * q;
    r0[q] = rr <= TY + 2u ? rr : TY + 2u;
    y0v[q] = wrap_row(c.y0 + r0[q], 2u, L);
  }
#pragma unroll
  for (int q = 0; q < N1; ++q) {
    const uint32_t rr = 2u + c.wave + W * q;
    r1[q] = rr <= TY + 1u ? rr : TY + 1u;
    y1v[q] = c.y0 + r1[q] - 2u;
  }
  uint32_t v0[N0][G][2], v1[N1][G][2];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const uint32_t g = c.lane + 64 * j;
#pragma unroll
    for (int q = 0; q < N0; ++q)
      stream3_group<TY, W, G, NEVER, 0, S % 6, (S + 1) % 6, (S + 2) % 6>(c, r0[q], y0v[q], za, g, v0[q][j][0], v0[q][j][1]);
#pragma unroll
    for (int q = 0; q < N1; ++q)
      stream3_group<TY, W, G, NEVER, 1, (S + 4) % 6, (S + 5) % 6, S % 6>(c, r1[q], y1v[q], zb, g, v1[q][j][0], v1[q][j][1]);
  }
  if (col0) {
#pragma unroll
    for (int q = 0; q < N0; ++q) {
      if (1u + c.wave + W * q > TY + 2u) break;
      int8_t* row = c.ring + ((S + 1) % 6) * PB + r0[q] * RB + 16;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint32_t g = c.lane + 64 * j;
        const uint2 v = make_uint2(v0[q][j][0], v0[q][j][1]);
        *reinterpret_cast<uint2*>(row + 8 * g) = v;
        if (g >= GPR - 2) *reinterpret_cast<uint2*>(row - 16 + 8 * (g - (GPR - 2))) = v;
        if (g < 2) *reinterpret_cast<uint2*>(row + L + 8 * g) = v;
      }
    }
  }
  if (col1) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      if (2u + c.wave + W * q > TY + 1u) break;
      const uint32_t roff = (zb * L + y1v[q]) * L;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const u32x2 w = {v1[q][j][0], v1[q][j][1]};
        __builtin_amdgcn_raw_buffer_store_b64(w, c.rdst, 8u * (c.lane + 64 * j), roff, 0);
      }
    }
  }
  if (do_load) c.put_plane((S + 3) % 6, nxt);
  __syncthreads();
}

template <int TY, int W, int G, bool NEVER>
__global__ __launch_bounds__(64 * W) void k_stream3d(const int8_t* __restrict__ src,
                                                     int8_t* __restrict__ dst, PhaseArgs a,
                                                     uint32_t H) {
  using X = Stream3Ctx<TY, W, G>;
  __shared__ __align__(16) int8_t lds[32 + 6 * X::PB];
  X c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(X::L * X::L * X::L), 0x00020000);
  c.rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(X::L * X::L * X::L), 0x00020000);
  c.ring = lds + 32;
  c.bound = reinterpret_cast<const uint32_t*>(lds);
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  c.U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  c.never4 = a.never4;
  c.y0 = blockIdx.x * TY;
  c.z0 = blockIdx.y * H;
  c.H = H;
  c.lane = threadIdx.x & 63;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x < 8) reinterpret_cast<uint32_t*>(lds)[threadIdx.x] = a.bound[threadIdx.x];
  for (uint32_t k = 0; k < 3; ++k) {
    uint2 v[X::RPW][G];
    c.get_plane(wrap_row(c.z0 + k, 2u, X::L), v);
    c.put_plane(k, v);
  }
  __syncthreads();
  const uint32_t steps = H + 3;
  for (uint32_t i0 = 0; i0 < steps; i0 += 6) {
    stream3_step<TY, W, G, NEVER, 0>(c, i0 + 0);
    stream3_step<TY, W, G, NEVER, 1>(c, i0 + 1);
    stream3_step<TY, W, G, NEVER, 2>(c, i0 + 2);
    stream3_step<TY, W, G, NEVER, 3>(c, i0 + 3);
    stream3_step<TY, W, G, NEVER, 4>(c, i0 + 4);
    stream3_step<TY, W, G, NEVER, 5>(c, i0 + 5);
  }
}

// 3D streaming shapes: tile.x == L == 512*G, tile.y = TY, tile.z = H, threads = 64*W.
bool stream3d_shape(const Lat& lat, const Tile& tile) {
  if (lat.J != nullptr || lat.d != 3) return false;
  if ((uint32_t)tile.x != lat.L || (lat.L != 512 && lat.L != 1024)) return false;
  const bool ok_shape = (tile.y == 8 && (tile.threads == 640 || tile.threads == 320)) ||
                        (tile.y == 16 && (tile.threads == 576 || tile.threads == 384)) ||
                        (tile.y == 32 && tile.threads == 704 && lat.L == 512);
  return ok_shape && lat.L % (uint32_t)tile.y == 0 && tile.z >= 4 && tile.z % 2 == 0 &&
         lat.L % (uint32_t)tile.z == 0;
}

template <int TY, int W, int G>
static hipError_t gostream3(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a,
                            bool never, uint32_t H, hipStream_t stream) {
  dim3 grid(lat.L / TY, lat.L / H);
  if (never)
    hipLaunchKernelGGL((k_stream3d<TY, W, G, true>), grid, dim3(64 * W), 0, stream, src, dst, a, H);
  else
    hipLaunchKernelGGL((k_stream3d<TY, W, G, false>), grid, dim3(64 * W), 0, stream, src, dst, a, H);
  return hipGetLastError();
}

hipError_t launch_stream3d(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           const Tile& tile, hipStream_t stream) {
  if (!stream3d_shape(lat, tile)) return hipErrorInvalidValue;
  const uint32_t H = (uint32_t)tile.z;
  if (lat.L == 512) {
    if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 1>(lat, src, dst, a, never, H, stream);
    if (tile.y == 8) return gostream3<8, 5, 1>(lat, src, dst, a, never, H, stream);
    if (tile.y == 16 && tile.threads == 576) return gostream3<16, 9, 1>(lat, src, dst, a, never, H, stream);
    if (tile.y == 16) return gostream3<16, 6, 1>(lat, src, dst, a, never, H, stream);
    return gostream3<32, 11, 1>(lat, src, dst, a, never, H, stream);
  }
  if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 2>(lat, src, dst, a, never, H, stream);
  if (tile.y == 8) return gostream3<8, 5, 2>(lat, src, dst, a, never, H, stream);
  if (tile.y == 16 && tile.threads == 576) return gostream3<16, 9, 2>(lat, src, dst, a, never, H, stream);
  return gostream3<16, 6, 2>(lat, src, dst, a, never, H, stream);
}

}  // namespace spin
