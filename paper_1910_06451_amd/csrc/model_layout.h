// Layout of the prepared support set ("model blob"), shared by the prepare
// kernel and the scoring kernels. The blob is private to the library.
//
//   [0, 256)          header: f_const (float) = (#fixed points / M) * sum_i alpha_i
//   fp32 MFMA tiles   ntiles x kTileFloats(Mp) floats, one tile = 16 supports:
//                       A[k][s][m] (k < 4, s < 16, m < Mp): -gamma * p'_{s,m,k} for k < 3, 1 for k = 3
//                       C[g][m][r] (g < 4, m < Mp, r < 4):  gamma/2 ||p'_{4g+r,m}||^2
//                       W[s]       (s < 16):                alpha_s / M
//   VALU rows         S_pad x Mp x 4 floats: (-gamma x', -gamma y', -gamma z', gamma/2 ||p'||^2), W in the
//                     fp32 tiles
//   BF16 tiles        ntiles x kTileBf16Bytes(Mp) bytes (see score kernels)
//
// Only the Mm moving control points (frame >= 1) are stored, in slots
// 0..Mm-1; slots Mm..Mp-1 and padded supports hold A = (0,0,0,1), C = 0,
// W = 0, which contribute exactly nothing. Points fixed to the base frame
// coincide for every pair of configurations, so each contributes exactly
// K_RQ = 1 per pair and is folded into f_const.
#pragma once

#include <cstdint>

namespace fastron {

constexpr int kTile = 16;
constexpr int64_t kHeaderBytes = 256;

inline int mp_of(int M) { return (M + 3) & ~3; }
inline int64_t ntiles_of(int64_t S) { return (S + kTile - 1) / kTile; }

__host__ __device__ constexpr int64_t tile_floats(int Mp) { return 64 * Mp + 16 * Mp + 16; }
__host__ __device__ constexpr int64_t tile_c_offset(int Mp) { return 64 * Mp; }
__host__ __device__ constexpr int64_t tile_w_offset(int Mp) { return 80 * Mp; }

// BF16 tile: per m, an A operand of 16 supports x 32 k (bf16) = 1 KB that also
// carries c_s (three bf16 parts); W is read from the fp32 tile.
__host__ __device__ constexpr int64_t tile_bf16_bytes(int Mp) { return (int64_t)Mp * 16 * 32 * 2; }

inline int64_t fp32_tiles_offset() { return kHeaderBytes; }
inline int64_t valu_offset(int64_t S, int M) { return kHeaderBytes + ntiles_of(S) * tile_floats(mp_of(M)) * 4; }
inline int64_t bf16_offset(int64_t S, int M) {
  return valu_offset(S, M) + ntiles_of(S) * kTile * (int64_t)mp_of(M) * 4 * 4;
}
inline int64_t model_bytes(int64_t S, int M) {
  return bf16_offset(S, M) + ntiles_of(S) * tile_bf16_bytes(mp_of(M));
}

}  // namespace fastron
