"""MI355X-native matrix-free (Id - J Lambda T) operator and Jacobi-Krylov solvers."""
