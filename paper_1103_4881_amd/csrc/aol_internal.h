// Internal structures shared by the host library and the kernels.
//
// A downscale tile covers TRx x TRy repetitions (Sec. III-A: one repetition
// is one elementary task consuming a packet of q pixels and emitting p).
// Each axis' filter is recast as a band of 16-output blocks: output block b
// of a tile reads a contiguous window of input elements, cut into 16-byte
// chunks, and that window times the block's coefficients is one small dense
// matrix product on the matrix cores. The host builds, per axis, the window
// of every block and the coefficient operand for every (block, K-step) in
// the exact per-lane order the MFMA instruction consumes it.
#pragma once
#include <stdint.h>

namespace aol {

constexpr int kMaxNB = 32;     // output blocks of 16 per tile and axis
constexpr int kLanes = 64;     // wavefront width
constexpr int kChunkBytes = 16;

enum Elem : int32_t { kU8 = 0, kBF16 = 1, kFP16 = 2 };

// One axis of one filter at one tile size. Device resident (read through
// the scalar cache).
struct alignas(16) AxisBand {
  int32_t p, q, taps, tr;   // ratio p/q, taps, repetitions per tile
  int32_t n_out;            // p * tr outputs per full tile
  int32_t nblk;             // ceil(n_out / 16)
  int32_t span;             // union window length of one repetition
  int32_t s_min;            // union window start relative to q*r
  int32_t delta;            // offset of the tile window inside its first chunk
  int32_t chunk_elems;      // elements per 16-byte chunk (16 for u8, 8 for 16-bit)
  int32_t nchunks;          // chunks touched by any K-step of a full tile
  int32_t split;            // u8: coefficients carried as lo + 128*hi operands
  int32_t chunk0[kMaxNB];   // first chunk of block b's window
  int32_t nk[kMaxNB];       // K-steps (4 chunks each) of block b
  int32_t frag[kMaxNB];     // first fragment of block b (64 lanes x 16 B each)
  int32_t bias[kMaxNB * 16];  // u8: 128*sum(c[phi]) + 128 for each output of the tile
};

struct PlaneArg {
  const void* in;
  void* out;
  int64_t in_pitch, out_pitch;    // elements
  int64_t in_fstride, out_fstride;  // elements between frames
  int32_t h, w, mh, mw;           // input and output sizes
  int32_t rx, ry;                 // repetitions along a line / along a column
  int32_t tiles_x, tiles_y;
  int32_t tile_base;              // first tile of this plane inside a frame
  int32_t vec_in, vec_out;        // 1 if rows allow 16-byte loads / full-width stores
};

constexpr int kMaxPlanes = 4;

struct FusedArgs {
  PlaneArg pl[kMaxPlanes];
  int32_t n_planes, n_frames;
  int32_t tiles_per_frame;
  int32_t total_tiles;
  const AxisBand* hb;
  const AxisBand* vb;
  const void* hfrag;   // uint8x16 per lane, per fragment
  const void* vfrag;
  int32_t zpitch;      // elements per Z^T row in LDS
  int32_t zrows;       // Z^T rows (tile z-columns, multiple of 16)
  int32_t z_mblocks;   // 16-row blocks of z the horizontal pass computes per full tile
};

}  // namespace aol
