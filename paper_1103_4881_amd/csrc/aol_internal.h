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
constexpr int kMaxK = 4;       // K-steps (of 4 chunks) per output block
constexpr int kLanes = 64;     // wavefront width
constexpr int kChunkBytes = 16;
constexpr int kWaves = 4;      // waves per workgroup of the fused kernel
constexpr int kMaxSlots = 12;  // 16-byte tile loads in flight per lane

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
  int32_t nfrag;            // fragments (64 lanes x 16 B) of the whole band, the zero one included
  int32_t zfrag;            // K-step index of an all-zero fragment (after the others)
  int32_t kmax;             // largest nk of the band
  int32_t ubias;            // u8: every output has the same bias (all phases' taps have one sum)
  int32_t chunk0[kMaxNB];   // first chunk of block b's window
  int32_t nk[kMaxNB];       // K-steps (4 chunks each) of block b
  int32_t frag[kMaxNB];     // first fragment of block b (64 lanes x 16 B each)
  int32_t wend[kMaxNB];     // end (exclusive) of block b's nonzero taps, tile-local elements
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

// Shared-memory layout of one workgroup (byte offsets).
struct LdsLayout {
  int32_t frag_h, frag_v;   // coefficient fragments of both axes
  int32_t bias_h, bias_v;   // int32 biases (u8)
  int32_t x;                // input tile, xrows x xpitch bytes
  int32_t z;                // intermediate, transposed: zrows x zpitch elements (hi, then lo)
  int32_t total;
};

struct FusedArgs {
  PlaneArg pl[kMaxPlanes];
  int32_t n_planes, n_frames;
  int32_t tiles_per_frame;
  int32_t total_tiles;
  const AxisBand* hb;
  const AxisBand* vb;
  const void* hfrag;   // uint8x16 per lane, per fragment
  const void* vfrag;
  LdsLayout lds;
  int32_t zpitch;      // elements per Z^T row in LDS
  int32_t zrows;       // Z^T rows (tile z-columns, multiple of 16)
  int32_t z_mblocks;   // 16-row blocks of z the horizontal pass computes per full tile
  int32_t xpitch;      // bytes per input-tile row in LDS
  int32_t xchunks;     // 16-byte chunks per input-tile row (full tile)
  int32_t rows_per_load;  // input-tile rows one wave-wide load covers (64 / xchunks)
  int32_t load_rounds;    // rounds of prefetch slots that stage one full input tile
  int32_t walk;           // tile order inside a plane: 0 row-major, 1 column-major
};

constexpr int kBandThreads = 1024;     // threads of a band-kernel workgroup (16 waves)
constexpr int kBandLoadThreads = 512;  // waves 0-7 stream input lines into LDS, waves 8-15 compute
constexpr int kBandMaxSlots = 8;       // 16-byte chunks per loading lane and staged step
// The horizontal pass is cut into at least 16 shares (one or two per compute
// wave, and the loading waves' where they take shares), each taking one block
// position of the 16-repetition period, so a filter with more positions
// (p > 16) does not use the band kernel.
constexpr int kBandMinHShares = 16;

// One plane or video stream of the band kernel (device resident). A
// workgroup owns a column band of `xreps` repetitions (the full width when it
// fits) and walks a segment of `seg` repetitions down the plane.
struct BandStream {
  int32_t h, w, mh, mw;    // input and output sizes
  int32_t rx, ry;          // repetitions along a line / down the plane
  int64_t in_pitch, out_pitch;  // elements
  int32_t ptr;             // index of the input pointer in the pointer table (output follows)
  int32_t xreps;           // repetitions per column band (multiple of 16)
  int32_t nbh;             // 16-column blocks of a full band
  int32_t nch;             // 16-byte chunks staged per input line of a full band
  uint32_t nch_magic;      // ceil(2^32 / nch)
  int32_t seg;             // repetitions per segment (multiple of 16)
  int32_t ring;            // intermediate lines kept (a multiple of 16)
  int32_t rpitch;          // bytes between rows of the ring (of each half for the float form)
  int32_t zhalf;           // float form: bytes from the hi ring to the lo ring
  int32_t xpitch;          // bytes between staged lines
  // LDS byte offsets. The two staging buffers of 16 lines sit at the same
  // place for every stream of a launch (buffer 1 at lds_x + xbuf, xbuf from
  // the widest stream), apart from every stream's coefficients and ring, so
  // the next unit's first lines can be staged while a unit finishes.
  int32_t lds_x, lds_z, lds_fh, lds_fv, lds_bh, lds_bv;
  int32_t vec_in;          // line length a multiple of one chunk and pitch chunk aligned
  int32_t vec_out;         // 4 or 2: the larger of them dividing the output pitch (elements), else 0
  int32_t xbuf;            // bytes from staging buffer 0 to buffer 1 (the same for every stream of a launch)
  int32_t lds_vt;          // LDS byte offset of the vertical block table (64 entries, then 64 window ends)
  const AxisBand* hb;      // one period (16 repetitions) of each axis
  const AxisBand* vb;
  const void* hfrag;
  const void* vfrag;
  const void* vtab;        // vertical block table (copied into LDS at lds_vt)
};

// One unit of work of one frame (a column band of a stream and a segment
// of repetitions down it) with its geometry, computed on the host.
struct BandUnit {
  int32_t stream, ptr;     // stream, its entry in the pointer table
  int32_t zrow0, Lz;       // input lines [zrow0, zrow0 + Lz) the unit reads (before the wrap)
  int32_t M, NBV;          // steps of 16 lines, vertical output blocks
  int32_t a0;              // first input column of the staged band lines (before the wrap)
  int32_t orow0, ocol0;    // first output row and column
  int32_t row_end, col_end;  // output rows and columns end (exclusive, inside the plane)
  int32_t nbh;             // 16-column output blocks
  int32_t pad[4];
};

struct BandLaunch {
  const BandStream* streams;
  const BandUnit* units;         // the units of one frame
  // Unit ids (frame * units_per_frame + unit) grouped by workgroup:
  // workgroup g takes order[first[g]], ..., order[first[g + 1] - 1], in turn.
  // NULL: the kernel deals the frames' units to the workgroups in rounds.
  const int32_t* order;
  const int32_t* first;
  int32_t units_per_frame, n_frames, total_units;
  int32_t wg0, ngroups;          // the launch's workgroups [wg0, wg0 + ngroups) run these units
  int32_t grouped;               // rounds over frame-major items, the slots of one XCD consecutive
  int32_t aligned;               // every pointer 16-byte aligned (inputs) / 16-byte (outputs)
  void* const* ptr_table;        // device [in, out] pointer per stream, or NULL: use ptrs below
  const void* ptrs[2 * kMaxPlanes];
  int64_t fstride[2 * kMaxPlanes];  // elements between frames (in, out) per stream
};

}  // namespace aol
