// Planning helpers shared by the entry points: workspace layout, kernel keys, kernel choice.
#pragma once

#include <cstddef>

#include "../../include/bsvd.h"
#include "common.hpp"

namespace bsvd {

// Bump allocator for laying out one call's workspace (256-byte aligned blocks).
struct Arena {
    size_t off = 0;
    size_t alloc(size_t bytes, size_t align = 256) {
        off = (off + align - 1) & ~(align - 1);
        const size_t r = off;
        off += bytes;
        return r;
    }
};

enum { JK_WAVE = 0, JK_LDS = 1 };

struct JKey {
    int kind = 0, a = 0, b = 0;
    bool operator<(const JKey &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (a != o.a) return a < o.a;
        return b < o.b;
    }
};

struct QKey {
    int nb = 0, seg = 0, kr = 0;
    bool operator<(const QKey &o) const {
        if (nb != o.nb) return nb < o.nb;
        if (seg != o.seg) return seg < o.seg;
        return kr < o.kr;
    }
};

// Kernel choice for an M x N working matrix (M >= N): the wavefront-resident kernel when the
// matrix and its V fit one wave's registers, else the LDS-resident kernel.
inline int choose_jacobi(int dtype, int M, int N, unsigned flags, JKey *key) {
    int a = 0, b = 0;
    const bool wave_ok = jacobi_wave_supported(dtype, M, N, &a, &b);
    int la = 0, lb = 0;
    const bool lds_ok = jacobi_lds_supported(dtype, M, N, &la, &lb);
    if (flags & BSVD_SVD_FORCE_WAVE) {
        if (!wave_ok) return BSVD_EUNSUP;
        *key = JKey{JK_WAVE, a, b};
    } else if (flags & BSVD_SVD_FORCE_LDS) {
        if (!lds_ok) return BSVD_EUNSUP;
        *key = JKey{JK_LDS, la, lb};
    } else if (wave_ok) {
        *key = JKey{JK_WAVE, a, b};
    } else if (lds_ok) {
        *key = JKey{JK_LDS, la, lb};
    } else {
        return BSVD_EUNSUP;
    }
    return BSVD_OK;
}

}  // namespace bsvd
