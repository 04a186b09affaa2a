"""Plain FP64 CPU oracle of the coupled LB-MPCD step.  TEST INFRASTRUCTURE ONLY."""
