"""Seeded synthetic inputs (breathing phantoms, random volumes, storage
casts) shared by the oracle tests and the HIP path. No TNLM arithmetic."""
from .breathing import (WORKLOADS, Workload, breathing_phantom, clean_phase,
                        quantise, random_volumes, scaled_phantom,
                        streak_field, to_bf16_bits, bf16_bits_to_f32,
                        workload_inputs)

__all__ = ["WORKLOADS", "Workload", "breathing_phantom", "clean_phase",
           "quantise", "random_volumes", "scaled_phantom", "streak_field",
           "to_bf16_bits", "bf16_bits_to_f32", "workload_inputs"]
