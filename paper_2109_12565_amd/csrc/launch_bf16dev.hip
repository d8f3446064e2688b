// Kernels of one storage type (instantiated here, dispatched from tlb.hip).
#include "launch_impl.hpp"

template struct tlbh::Launcher<tlbk::StoreBF16Dev>;
