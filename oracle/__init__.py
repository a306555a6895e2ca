"""CPU oracle of the FRNN graph.  Test infrastructure only (see oracle.py)."""
