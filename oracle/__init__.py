"""CPU oracle of octree background modelling (test infrastructure only)."""
