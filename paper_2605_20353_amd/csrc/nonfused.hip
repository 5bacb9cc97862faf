// Kernels of the non-fused sampled gradient (Sec. 3.1.2, the form the fused
// sampling-MTTKRP improves on): k_loss_grad built to draw the samples and
// write the sampled tensor Y~ (SRC = 2: coordinates and y = w f'(x, m), the
// factor rows gathered once for m), and built to read such a tensor and
// scatter its MTTKRP (SRC = 3: the factor rows gathered a second time).
// Their own translation unit, so that they build in parallel with the fused
// kernels; the host side is gcp_sample_y / gcp_mttkrp in loss_grad.hip.
#include "lg_kernels.hpp"

namespace gcp {

template <typename T>
LGKernel<T> pick_kernel_nonfused(int d, int src, int lanes, int vec)
{
    if (src == 2) {
        if (d == 3) return pick_shape<T, 3, 2>(lanes, vec);
        if (d == 4) return pick_shape<T, 4, 2>(lanes, vec);
        return pick_shape<T, 0, 2>(lanes, vec);
    }
    if (src == 3) {
        if (d == 3) return pick_shape<T, 3, 3>(lanes, vec);
        if (d == 4) return pick_shape<T, 4, 3>(lanes, vec);
        return pick_shape<T, 0, 3>(lanes, vec);
    }
    return nullptr;
}

template LGKernel<float> pick_kernel_nonfused<float>(int, int, int, int);
template LGKernel<double> pick_kernel_nonfused<double>(int, int, int, int);

}  // namespace gcp
