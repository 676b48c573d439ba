// merge_internal.hpp -- workspace of the sector track merger (not ABI).
#pragma once
#include "internal.hpp"

namespace tpcca {

struct MergeWs {
  int64_t T;               // segments
  int64_t H;               // their hits (= hits of the merged output)
  int S, NW, R;            // sectors, wedges per side, pad rows
  Model m;                 // field, sin phi limit, cluster variances
  float chi2_merge, merge_dist;
  float ca, sa;            // cos and sin of the turn between adjacent wedges
  // segments (the tracking output) and the clusters their hit ids index
  const uint8_t* sector;
  const float* x_ref;
  const float* p;          // [T][5]
  const float* cov;        // [T][15]
  const float* chi2;
  const int32_t* ndf;
  const int32_t* hit_off;  // [T + 1]
  const uint32_t* hit_id;
  const float* cx;
  const float* cy;
  const float* cz;
  const int16_t* crow;
  int64_t NC;
  const int32_t* slice;    // [T] time-frame slice of each segment, or null (one event)
  int nsl;                 // slices of the frame (1 for one event): the lists are by (sector, slice)
  int prune;               // 1: the window is shorter than half a slice, so only segments of the
                           // same or a neighbouring slice can pass it
  // work
  float* ex;               // [T][24]: exit plane, state, covariance (if the exit transport succeeded)
  float4* first;           // [T] innermost hit (x, y, z, row bits)
  float4* last;            // [T] outermost hit (x, y, z, row bits)
  uint32_t* flags;         // [T] bit 0: exit state valid
  uint32_t* sec_cnt;       // [S nsl + 1] segments per (sector, slice), then offsets
  uint32_t* sec_cur;       // [S nsl] fill counts (from zero)
  uint32_t* sec_list;      // [T] segment indices by (sector, slice)
  unsigned long long* best_in;   // [T] (chi2 bits << 32) | inner partner, or ~0
  unsigned long long* best_out;  // [T] (chi2 bits << 32) | outer partner, or ~0
  int32_t* link;           // [T] outer partner or -1
  int32_t* inner;          // [T] inner partner or -1
  float4* zrec;            // [T] srec with every list of at most kZSort records sorted by z
  uint32_t* zlist;         // [T] sec_list in the same order
  uint8_t* zsorted;        // [S nsl] 1: the list is sorted by z
  float4* srec;            // [T] by (sector, slice): outermost hit (x, y, z), (slice << 9 | last row << 1 | exit valid) bits
  uint32_t* emit;          // [T + 1] output tracks of the chain headed by a segment -> offsets
  uint32_t* hemit;         // [T + 1] hits of those tracks -> offsets
  int32_t* head;           // [T] the head of each segment's chain
  uint32_t* tpos;          // [T] a segment's place in its chain
  uint32_t* hpos;          // [T] hits of the chain's segments before it
  uint32_t* nseg;          // [T] segments of the chain (at its head)
  uint32_t* rlist;         // [T] heads of chains of two or more segments
  float* rec;              // [T][24]: merged refit of a chain head (x_ref, p, cov, chi2)
  uint32_t* err;           // [4]: error bits, output tracks, output hits, chains to refit
  uint32_t* scan_part;     // [2 (T / 1024 + 2)] partial sums of the offset scans
  // outputs (device)
  uint8_t* o_sector;
  float* o_x_ref;
  float* o_p;
  float* o_cov;
  float* o_chi2;
  int32_t* o_ndf;
  int32_t* o_hit_off;
  uint32_t* o_hit_id;
  int32_t* o_link;         // optional [T]
};

hipError_t run_merge(const MergeWs& w, hipStream_t st);

}  // namespace tpcca
