"""Seeded synthetic input generators (no part of the regression method)."""
from .frames import (CONFIGS, make_config, make_frame, make_training_batch, random_frame,
                     small_integer_frame)

__all__ = ["CONFIGS", "make_config", "make_frame", "make_training_batch", "random_frame", "small_integer_frame"]
