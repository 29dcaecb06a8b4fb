"""CPU oracle of the ecological world step: test infrastructure only.

`oracle.oracle` wraps the C oracle (eco_oracle.c); `oracle.spec` is an
independent pure-Python statement of the same rules for tiny worlds.  Nothing in
the product package imports this package.
"""
