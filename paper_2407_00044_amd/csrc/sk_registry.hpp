// Registry of the compiled kernel instantiations (one per input type,
// operand layouts and tile shape), filled at library load time.
#pragma once

namespace sk {

struct KernelEntry {
  int dt, la, lb, bm, bn, wgm;
  int nt;           // threads per workgroup
  const void* fn;   // host handle of the __global__ function
};

// Adds an entry; called from static initialisers of the instantiation units.
bool register_kernel(const KernelEntry& e);

}  // namespace sk
