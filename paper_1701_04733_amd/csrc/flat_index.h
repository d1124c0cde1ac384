// Row / column of a flat element index in the elementwise kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace btas {

// (i, j) = (e / n, e % n) for 0 <= e < total = rows * n.  A 32-bit division
// when the matrix has fewer than 2^31 elements (every matrix up to
// 46340 x 46340): 64-bit division is a long instruction sequence and these
// kernels are otherwise only loads and stores.
__device__ __forceinline__ void flat_to_rc(long e, int n, long total, long& i, long& j) {
    if (total < (1L << 31)) {
        const unsigned q = (unsigned)e / (unsigned)n;
        i = q;
        j = e - (long)q * n;
    } else {
        i = e / n;
        j = e - i * n;
    }
}

}  // namespace btas
