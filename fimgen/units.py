"""Unit conversions to SI (everything inside the library and oracle is SI)."""
PSI = 6894.757293168          # Pa
MD = 9.869233e-16             # m^2 (millidarcy)
DAY = 86400.0                 # s
CP = 1.0e-3                   # Pa s (centipoise)
GRAV = 9.80665                # m/s^2
