"""FP64 CPU oracle of the explicit casting step. TEST INFRASTRUCTURE ONLY."""
