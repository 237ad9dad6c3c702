// Host-side helpers of the grouped launchers (kernels_*.hip): tables of
// per-problem arguments passed by value to one launch whose blockIdx.z picks
// the problem (GroupTab, internal.h).
#pragma once

#include "internal.h"

namespace topo {

template <class A>
inline GroupTab<A> group_tab(int G, const A *a) {
  GroupTab<A> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i];
  return t;
}
inline GroupTab<double *> group_partials(int G, const Reducer *red) {
  GroupTab<double *> t{};
  for (int i = 0; i < G; ++i) t.v[i] = red[i].partials;
  return t;
}
template <class A>
inline GroupTab<const int *> group_skips(int G, const A *a) {
  GroupTab<const int *> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i].skip;
  return t;
}
inline bool group_ok(int G) { return G >= 1 && G <= kMaxGroup; }

}  // namespace topo
