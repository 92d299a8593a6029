// hg_netrec.h -- building one net's record (w, lambda, Lambda bits, S bits)
// from its pin counts with a group of G lanes (G in {4,8,16,32,64}).
//
// Lane gl of the group handles blocks gl, gl+G, ...; the bitsets come from
// two wave ballots per chunk of G blocks (Phi > 0 and Phi == 1).  Every lane
// ends up holding the record word with index gl, so the record is written
// with one coalesced store per lane.
#pragma once

#include "hg_device.h"

namespace hg {

struct NetBits {
  int lambda;
  unsigned word;   // record word with index = lane-in-group (valid for 1 <= gl < 2+2W)
};

// get(i) -> Phi(e,i).  The first MC chunks' counts are loaded up front,
// unconditionally (indices past k clamped, values masked), so that their
// loads are in flight together; further chunks are read one at a time.
template <int G, int MC, typename Get>
__device__ __forceinline__ NetBits net_bits_mc(int k, int gl, Get get) {
  const int wk = bit_words(k);
  const int shift = (G == kWave) ? 0 : (lane_id() / G) * G;
  const unsigned long long gmask = (G == kWave) ? ~0ull : ((1ull << (G % kWave)) - 1);
  NetBits r;
  r.lambda = 0;
  r.word = 0;
  const int nchunks = (k + G - 1) / G;
  int cvs[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) {
    const int i = c * G + gl;
    cvs[c] = get(i < k ? i : k - 1);
  }
#pragma unroll
  for (int c = 0; c < MC; ++c)
    if (!(c < nchunks && c * G + gl < k)) cvs[c] = 0;
  for (int c = 0; c < nchunks; ++c) {
    int i = c * G + gl;
    int cv = 0;
    if (c < MC) {
#pragma unroll
      for (int x = 0; x < MC; ++x)
        if (x == c) cv = cvs[x];
    } else if (i < k) {
      cv = get(i);
    }
    unsigned long long nz = (__ballot(cv > 0) >> shift) & gmask;
    unsigned long long one = (__ballot(cv == 1) >> shift) & gmask;
    r.lambda += __popcll(nz);
    if (G <= 32) {                    // chunk c fills bits [c*G % 32, +G) of word c*G/32
      const int wd = (c * G) >> 5, sh = (c * G) & 31;
      if (gl == 2 + wd) r.word |= (unsigned)nz << sh;
      if (gl == 2 + wk + wd) r.word |= (unsigned)one << sh;
    } else {
      int j0 = 2 * c;
      if (gl == 2 + j0) r.word = (unsigned)nz;
      if (gl == 3 + j0) r.word = (unsigned)(nz >> 32);
      if (gl == 2 + wk + j0) r.word = (unsigned)one;
      if (gl == 3 + wk + j0) r.word = (unsigned)(one >> 32);
    }
  }
  if (gl == 1) r.word = (unsigned)r.lambda;
  return r;
}

// Record bits of one net with G lanes: as many up-front loads as k has
// chunks of G blocks (1, 2, 4, or 8 and more).  k is the same for every lane
// of the wavefront, so the branch does not diverge.
template <int G, typename Get>
__device__ __forceinline__ NetBits net_bits(int k, int gl, Get get) {
  const int nchunks = (k + G - 1) / G;
  if (nchunks <= 1) return net_bits_mc<G, 1>(k, gl, get);
  if (nchunks <= 2) return net_bits_mc<G, 2>(k, gl, get);
  if (nchunks <= 4) return net_bits_mc<G, 4>(k, gl, get);
  return net_bits_mc<G, 8>(k, gl, get);
}

// Write a whole record (w in word 0, zero padding); needs G >= record words,
// which holds for the group sizes chosen per k (G >= 4 = words for k <= 32,
// G = 64 >= 32 words otherwise).
__device__ __forceinline__ void write_netrec(unsigned* rec, int gl, int w, const NetBits& b,
                                             int k) {
  const int wk = bit_words(k);
  const int rw = net_words(k);
  if (gl < rw) {
    unsigned val = 0;
    if (gl == 0) val = (unsigned)w;
    else if (gl < 2 + 2 * wk) val = b.word;
    rec[gl] = val;
  }
}

// Write net e's entry of the compact Lambda/S view (NetView) from the record
// words held by the group's lanes (lane 2.. holds Lambda, then S).  All lanes
// of the group must call it.
__device__ __forceinline__ void write_view(unsigned* view, long long e, int view_kind, int gl,
                                           const NetBits& b) {
  const unsigned next = __shfl(b.word, lane_id() + 1);   // the word of lane gl + 1
  if (view_kind == kView16) {
    if (gl == 2) view[e] = (b.word & 0xffffu) | (next << 16);
  } else if (view_kind == kView32) {
    if (gl == 2 || gl == 3) view[e * 2 + (gl - 2)] = b.word;
  } else if (view_kind == kView64) {
    if (gl >= 2 && gl < 6) view[e * 4 + (gl - 2)] = b.word;
  }
}

}  // namespace hg
