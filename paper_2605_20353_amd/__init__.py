"""MI355X (gfx950) library for the sampled stochastic gradient of GCP tensor
decomposition (Myers & Phipps, arXiv 2605.20353): stratified sampling, fused
model values / loss derivative / sampled MTTKRP, Adam, and batched GCP-FedAdam,
as hand-written HIP kernels behind the C ABI in include/gcp.h.
"""
from ._lib import (  # noqa: F401
    GCPError, SampleParams, Tile, SparseTensor, DenseTensor,
    gcp_tensor_create, gcp_tensor_create_dense, gcp_tensor_destroy, gcp_tensor_reserve, gcp_device_status,
    gcp_sample, gcp_loss_grad, gcp_adam_step, lib,
)
from .autograd import GCPLoss, KruskalModel, gcp_loss  # noqa: F401,E402
from .fedadam import Batched, FedAdam, FedConfig, FedTile, Plain  # noqa: F401,E402
from .solver import SolverConfig, SolverResult, gcp_adam  # noqa: F401,E402
