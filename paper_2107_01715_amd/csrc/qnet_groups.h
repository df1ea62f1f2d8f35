// conv1 by sibling groups on the layer-by-layer Q-network path.
#pragma once
#include "bcts_internal.h"

namespace bcts {

// The sibling groups of a chunk: groups[0..n) cover the chunk's items
// exactly (plan-global first items; item_base is the chunk's first item).
struct ChunkGroups {
  const FusedGroup* groups;
  int n;
  long long item_base;
};

// launch_qnet, with conv1 computing the channels a group's stacks share
// (0..2) once per group; results equal launch_qnet's bit for bit.  n == 0
// runs conv1 stack by stack, as launch_qnet does.
void launch_qnet_groups(int prec, const QnetDev& q, const ItemDesc* desc, long long n_items, const ChunkGroups& cg,
                        void* ws, float* V, float* q0, hipStream_t s, hipEvent_t* ev = nullptr);

}  // namespace bcts
