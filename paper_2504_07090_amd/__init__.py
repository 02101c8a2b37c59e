"""MI355X-native visibility simulation and gradient hot path (BayesLIM forward model).

Import submodules explicitly: ``workload`` (seeded synthetic inputs) has no
GPU dependency; ``vis`` loads the HIP library and fails loudly without it.
"""
__all__ = ["workload", "vis", "serve"]
