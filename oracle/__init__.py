"""CPU oracle of the parallel event-chain sweep -- test infrastructure only."""
