"""MI355X-native MAX-MIN Ant System hot path (tour construction by weighted
reservoir sampling over candidate lists, plus the pheromone update).

Importing the package loads nothing native; `paper_2003_11902_amd.mmas` loads
the HIP library and fails loudly if it is not built.
"""
__all__ = ["instances", "mmas"]
