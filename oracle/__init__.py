"""CPU oracle of the CoG background subtractor -- test infrastructure only."""
