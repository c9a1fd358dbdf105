// uf_cached.h -- union for passes that unite many pairs which are mostly connected already (the pentachoron passes
// of isovolume and vortex surface tracking).
#pragma once

#include "common.h"

namespace ftk {

// Unite for passes in which most pairs are already connected: first a find through plain (cached, possibly stale)
// loads.  A stale parent is still an ancestor and sets only merge, so equal roots mean the pair is connected now;
// otherwise the coherent path (uf_unite) decides.
__device__ __forceinline__ unsigned uf_find_cached(const unsigned* parent, unsigned x) {
  unsigned p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

__device__ __forceinline__ void uf_unite_cached(unsigned* parent, unsigned a, unsigned b) {
  if (uf_find_cached(parent, a) == uf_find_cached(parent, b)) return;
  uf_unite(parent, a, b);
}

// Unions of every member of a group with its first member: r is the group's representative as last found (found
// from the first member, so an element of its set).  A member whose cached find reaches r is connected already;
// otherwise the coherent path unites them and r is found again.  Returns the representative for the next member
// (one find per member instead of two).
__device__ __forceinline__ unsigned uf_unite_into(unsigned* parent, unsigned r, unsigned b) {
  if (uf_find_cached(parent, b) == r) return r;
  uf_unite(parent, r, b);
  return uf_find_cached(parent, r);
}

}  // namespace ftk
