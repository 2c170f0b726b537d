"""Checks that pin the oracle to something other than itself: the explicit
graph of eqs. (25)-(31), Dijkstra shortest paths, brute-force path
enumeration, closed forms and free-space geometry."""
