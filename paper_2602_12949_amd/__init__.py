"""MI355X-native hot path of the Neural Irradiance Volume (Coomans, Nazzaro
et al., Eurographics 2026): fused per-pixel queries, on-GPU training and a
Monte Carlo irradiance estimator, behind the C interface of libniv.so."""
from .niv import NIV, McScene, Trainer, NivError, lib, FP32, FP16, BF16, PRECISIONS  # noqa: F401
